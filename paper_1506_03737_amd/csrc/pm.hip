// Particle kernels of liblpc: the fixed-point CIC deposit (Sec. 2.4 step 1, Sec. 4.2 "rounding down" to the cell),
// the CIC force gather fused with the COLA kick and drift (Sec. 2.4 step 4; Sec. 2.3 Eqs. 17-18), and the frame
// momentum removal / add-back (Sec. 2.3).
//
// Fixed point: per axis u = floor(x * (Nm 2^16 / L)) in FP64, reduced mod Nm 2^16; the cell is u >> 16 and the
// fraction f = u & 0xffff. The deposit adds prod_d (2^16 - f_d or f_d) to the 8 corners with 64-bit integer atomics,
// so every particle adds exactly 2^48 and the mesh does not depend on the order of the additions. The gather uses
// the same u, with weights f 2^-16 and 1 - f 2^-16 (exact in FP32), so it is the transpose of the deposit.
//
// The kernels are batched over the jobs (boxes) of a work table and launched with one workgroup per item (their
// loops stride over the grid, so any grid size is correct); an item is kNT particles of one box.
#include <hip/hip_runtime.h>

#include <cmath>

#include "lpc_kernels.h"

namespace lpc {
namespace kern {

namespace {

constexpr uint32_t kOne = 1u << kFracBits;
constexpr uint32_t kMask = kOne - 1u;

// Fixed-point coordinate of one axis; false if x is not finite or too far outside the box to convert.
// For a wrapped position, 0 <= x scale < Nm 2^16 <= 2^31, so floor is a 32-bit truncation (one conversion); the
// 64-bit floor and remainder are only taken for positions outside the box.
__device__ __forceinline__ bool fixed_coord(float x, double scale, int64_t period, uint32_t* cell, uint32_t* frac) {
  const double xs = static_cast<double>(x) * scale;
  uint32_t u32;
  if (xs >= 0.0 && xs < static_cast<double>(period)) {
    u32 = static_cast<uint32_t>(xs);
  } else {
    if (!(fabs(xs) < 4.0e18)) return false;  // also catches NaN
    int64_t u = static_cast<int64_t>(floor(xs)) % period;
    if (u < 0) u += period;
    u32 = static_cast<uint32_t>(u);
  }
  *cell = u32 >> kFracBits;
  *frac = u32 & kMask;
  return true;
}

// The three axes of a position at once: one branch for the common case (every axis inside the box) instead of one
// per axis; each branch a wave takes divergently costs the scalar unit an exec-mask save and restore.
__device__ __forceinline__ bool fixed_coord3(const float x[3], double scale, int64_t period, uint32_t c[3],
                                             uint32_t f[3]) {
  double xs[3];
  bool in = true;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    xs[d] = static_cast<double>(x[d]) * scale;
    in = in && xs[d] >= 0.0 && xs[d] < static_cast<double>(period);
  }
  if (in) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const uint32_t u = static_cast<uint32_t>(xs[d]);
      c[d] = u >> kFracBits;
      f[d] = u & kMask;
    }
    return true;
  }
  bool ok = true;
#pragma unroll
  for (int d = 0; d < 3; ++d) ok &= fixed_coord(x[d], scale, period, &c[d], &f[d]);
  return ok;
}

// a b for a < 2^33 and b <= 2^16 (a product of two axis weights times a third): one 32 x 32 -> 64 multiply-add for
// the low word and a 32-bit multiply for the high one.
__device__ __forceinline__ uint64_t mul_weight(uint64_t a, uint32_t b) {
  return static_cast<uint64_t>(static_cast<uint32_t>(a)) * b +
         (static_cast<uint64_t>(static_cast<uint32_t>(a >> 32) * b) << 32);
}

// t / d for t < 2^32 / d, with inv = ceil(2^32 / d) computed on the host (0 for d = 1): one high multiply.
__device__ __forceinline__ uint32_t fast_div(int t, uint32_t inv) {
  return inv ? __umulhi(static_cast<uint32_t>(t), inv) : static_cast<uint32_t>(t);
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

__global__ __launch_bounds__(kNT) void k_fill_i32(int* __restrict__ p, size_t count, int value) {
  const size_t stride = static_cast<size_t>(gridDim.x) * kNT;
  for (size_t i = static_cast<size_t>(blockIdx.x) * kNT + threadIdx.x; i < count; i += stride) p[i] = value;
}

// ---------------------------------------------------------------------------------------------------------------
// Tile sort. A box's mesh is cut into tiles of kTX x kTY x kTZ cells (the last tile of an axis may be narrower); a
// particle belongs to the tile of its floor cell, and within it to one of two buckets: interior, or boundary when its
// cell is in the last layer of the tile along any axis (only boundary particles can reach the next tile's cells).
// Bucket 2 t + boundary; the box's last bucket (2 ntx nty ntz) holds particles whose position is unusable.
// Key pass: bucket and rank among the bucket's particles. Scan: bucket starts. Scatter: copy each record to
// start[bucket] + rank. The order within a bucket is not deterministic, but nothing downstream depends on it: the
// deposit is integer and the other particle stages act per particle.

template <class J>
__device__ __forceinline__ int bucket_of(uint32_t cx, uint32_t cy, uint32_t cz, const J& job) {
  const int t = (static_cast<int>(cx / kTX) * job.nty + static_cast<int>(cy / kTY)) * job.ntz + static_cast<int>(cz / kTZ);
  const int nm = job.nm;
  const bool last = (cx % kTX == kTX - 1) || (cy % kTY == kTY - 1) || (cz % kTZ == kTZ - 1) ||
                    (static_cast<int>(cx) == nm - 1) || (static_cast<int>(cy) == nm - 1) ||
                    (static_cast<int>(cz) == nm - 1);
  return 2 * t + (last ? 1 : 0);
}

// Rank of each active thread among the threads of its workgroup with the same bucket g, with one counter atomic per
// distinct bucket in the workgroup: longer runs of one bucket in the sorted copy than a wave's (fewer partial cache
// lines written by the scatter). Wave runs of one bucket are merged through an LDS hash of the block's buckets
// (kRankSlots >= 2 kNT slots, linear probing, so an insert always finds a slot); LDS atomics give each run its offset
// in the block, and the leader thread of each slot takes the block's range from cnt. Called by all threads of the
// workgroup (it has barriers); sh holds 3 kRankSlots ints.
constexpr int kRankSlots = 2 * kNT;
__device__ int block_rank(int* __restrict__ cnt, int g, bool active, int* sh) {
  int* s_key = sh;
  int* s_cnt = sh + kRankSlots;
  int* s_base = sh + 2 * kRankSlots;
  for (int t = threadIdx.x; t < kRankSlots; t += kNT) {
    s_key[t] = -1;
    s_cnt[t] = 0;
  }
  __syncthreads();
  const int lane = __lane_id();
  const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  unsigned long long pending = __ballot(active);
  int slot = 0, local = 0;
  while (pending) {
    const int leader = __ffsll(static_cast<long long>(pending)) - 1;
    const int lg = __shfl(g, leader);
    const unsigned long long same = __ballot(active && g == lg);
    int sl = 0, off = 0;
    if (lane == leader) {
      sl = static_cast<int>((static_cast<unsigned>(lg) * 2654435761u) % kRankSlots);
      while (true) {
        const int prev = atomicCAS(s_key + sl, -1, lg);
        if (prev == -1 || prev == lg) break;
        sl = (sl + 1) % kRankSlots;
      }
      off = atomicAdd(s_cnt + sl, __popcll(same));
    }
    sl = __shfl(sl, leader);
    off = __shfl(off, leader);
    if (active && g == lg) {
      slot = sl;
      local = off + __popcll(same & below);
    }
    pending &= ~same;
  }
  __syncthreads();
  for (int t = threadIdx.x; t < kRankSlots; t += kNT)
    if (s_key[t] >= 0) s_base[t] = atomicAdd(cnt + s_key[t], s_cnt[t]);
  __syncthreads();
  const int rank = active ? s_base[slot] + local : 0;
  __syncthreads();  // sh is reused by the next call
  return rank;
}

__global__ __launch_bounds__(kNT) void k_tile_key(const SortJob* __restrict__ jobs, const int* __restrict__ offs,
                                                  int njob, int total, int* __restrict__ cnt, int* __restrict__ key,
                                                  int* __restrict__ rank, int* __restrict__ flags) {
  __shared__ int sh[3 * kRankSlots];
  for (int w = blockIdx.x; w < total; w += gridDim.x) {
    const int jb = __builtin_amdgcn_readfirstlane(find_job(to_const(offs), njob, w));
    const LPC_CONST SortJob& J = to_const(jobs)[jb];
    const int64_t n = J.n;
    const int64_t i = static_cast<int64_t>(xcd_remap(w - offs[jb], offs[jb + 1] - offs[jb])) * kNT + threadIdx.x;
    const bool active = i < n;
    int g = 0;
    if (active) {
      LPC_GLOBAL const float* pos = to_global(J.pos);
      const int64_t period = static_cast<int64_t>(J.nm) << kFracBits;
      float x[3];  // the three loads go out together
#pragma unroll
      for (int d = 0; d < 3; ++d) x[d] = pos[d * n + i];
      uint32_t c[3], f[3];
      bool ok = true;
#pragma unroll
      for (int d = 0; d < 3; ++d) ok &= fixed_coord(x[d], J.scale, period, &c[d], &f[d]);
      int b = 2 * J.ntx * J.nty * J.ntz;
      if (ok)
        b = bucket_of(c[0], c[1], c[2], J);
      else
        atomicOr(flags + kFlagNonfinite, 1);
      g = J.tbase + b;
    }
    const int r = block_rank(cnt, g, active, sh);
    if (active) {
      key[J.pbase + i] = g;
      rank[J.pbase + i] = r;
    }
  }
}

// Exclusive scan of cnt[0..count) into start[0..count] in three launches: block-local scans of kScanBlock elements
// (writing block totals), a scan of the block totals, and the add of each block's offset.
constexpr int kScanPer = 8;
constexpr int kScanBlock = kNT * kScanPer;

__device__ __forceinline__ int block_exclusive_scan(int v, int* sh, int* total) {
  // sh: kNT ints of LDS; Hillis-Steele over the workgroup
  const int tid = threadIdx.x;
  sh[tid] = v;
  __syncthreads();
  for (int off = 1; off < kNT; off <<= 1) {
    const int u = (tid >= off) ? sh[tid - off] : 0;
    __syncthreads();
    sh[tid] += u;
    __syncthreads();
  }
  const int incl = sh[tid];
  *total = sh[kNT - 1];
  __syncthreads();
  return incl - v;
}

__global__ __launch_bounds__(kNT) void k_scan_local(const int* __restrict__ cnt, int* __restrict__ start, int count,
                                                    int* __restrict__ block_sums) {
  __shared__ int sh[kNT];
  const int base = blockIdx.x * kScanBlock + threadIdx.x * kScanPer;
  int v[kScanPer];
  int sum = 0;
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) {
    v[k] = (base + k < count) ? cnt[base + k] : 0;
    sum += v[k];
  }
  int total;
  int run = block_exclusive_scan(sum, sh, &total);
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) {
    if (base + k < count) start[base + k] = run;
    run += v[k];
  }
  if (threadIdx.x == 0) block_sums[blockIdx.x] = total;
}

// One workgroup: exclusive scan of the block totals in place, and start[count] = the grand total.
__global__ __launch_bounds__(kNT) void k_scan_sums(int* __restrict__ block_sums, int nblocks, int* __restrict__ start,
                                                   int count) {
  __shared__ int sh[kNT];
  int carry = 0;
  for (int b0 = 0; b0 < nblocks; b0 += kNT) {
    const int b = b0 + threadIdx.x;
    const int v = (b < nblocks) ? block_sums[b] : 0;
    int total;
    const int ex = block_exclusive_scan(v, sh, &total);
    if (b < nblocks) block_sums[b] = carry + ex;
    carry += total;
  }
  if (threadIdx.x == 0) start[count] = carry;
}

__global__ __launch_bounds__(kNT) void k_scan_add(int* __restrict__ start, int count,
                                                  const int* __restrict__ block_sums) {
  const int base = blockIdx.x * kScanBlock;
  const int add = block_sums[blockIdx.x];
  for (int k = threadIdx.x; k < kScanBlock; k += kNT)
    if (base + k < count) start[base + k] += add;
}

// The sort's kernels (keys, scatter, unsort) give each XCD contiguous ranges of particles, so that the runs they
// write into one bucket mostly come from one XCD's L2: eighths of the range per XCD (xcd_remap) took the scatter from
// 0.53 to 0.52 ms and the unsort from 0.55 to 0.46 ms at 768^3; the scatter then takes XCD-contiguous chunks of 64
// items in turn (xcd_chunk_remap: 0.52 -> 0.48 ms; chunks of 256 the same, the key pass and the unsort no different).
// The gather/kick/drift and the frame momentum measured slower with eighths (1.11 -> 1.15 and 0.15 -> 0.17 ms; the
// gather 1.22 ms with chunks of 32) and keep consecutive items on consecutive XCDs.
// The scatter copies one array at a time (each load next to its store); issuing all of a particle's loads first
// measured slower (0.51 -> 0.54 ms).
__global__ __launch_bounds__(kNT) void k_scatter(const SortJob* __restrict__ jobs, const int* __restrict__ offs,
                                                 int njob, int total, const int* __restrict__ key,
                                                 const int* __restrict__ rank, const int* __restrict__ start) {
  for (int w = blockIdx.x; w < total; w += gridDim.x) {
    const int jb = __builtin_amdgcn_readfirstlane(find_job(to_const(offs), njob, w));
    const LPC_CONST SortJob& J = to_const(jobs)[jb];
    const int64_t n = J.n;
    const int64_t i =
        static_cast<int64_t>(xcd_chunk_remap(w - offs[jb], offs[jb + 1] - offs[jb], 64)) * kNT + threadIdx.x;
    if (i >= n) continue;
    const int64_t gi = J.pbase + i;
    const int64_t dst = static_cast<int64_t>(start[key[gi]]) + rank[gi] - J.pbase;
    LPC_GLOBAL const float* pos = to_global(J.pos);
    LPC_GLOBAL float* dpos = to_global(J.dpos);
#pragma unroll
    for (int d = 0; d < 3; ++d) dpos[d * n + dst] = pos[d * n + i];
    if (J.dvel) {
      LPC_GLOBAL const float* vel = to_global(J.vel);
      LPC_GLOBAL float* dvel = to_global(J.dvel);
#pragma unroll
      for (int d = 0; d < 3; ++d) dvel[d * n + dst] = vel[d * n + i];
    }
    if (J.dpsi1) {
      LPC_GLOBAL const float* p1 = to_global(J.psi1);
      LPC_GLOBAL const float* p2 = to_global(J.psi2);
      LPC_GLOBAL float* d1 = to_global(J.dpsi1);
      LPC_GLOBAL float* d2 = to_global(J.dpsi2);
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        d1[d * n + dst] = p1[d * n + i];
        d2[d * n + dst] = p2[d * n + i];
      }
    }
    to_global(J.dorig)[dst] = J.orig ? to_global(J.orig)[i] : static_cast<int>(i);
  }
}

// ---------------------------------------------------------------------------------------------------------------
// Tiled deposit: one workgroup per mesh tile. It reads the sorted particles of its own tile (both buckets) and the
// boundary buckets of the (up to 7) lower neighbour tiles, whose particles can reach its cells; accumulates the
// integer weights of the corners that fall inside its tile with 64-bit LDS atomics; and writes every cell of the
// tile once with plain stores (so the mesh needs no clearing and sees no global atomics). The up to 8 particle
// ranges are walked as one index space, so a workgroup needs few rounds of loads.
constexpr int kTileCells = kTX * kTY * kTZ;
// A cell's exact count C is a sum of corner weights of at most 2^48 each. With fewer than 2^16 particles reaching a
// tile, C < 2^64 cannot wrap its 64-bit sum and bit 63 tells whether C >= 2^63 (the headroom of a signed count).
// A tile reached by 2^16 or more particles also sums the weights' high parts T = sum(w >> 16), which cannot wrap;
// with the wrapped sum S = C mod 2^64, R = S - T 2^16 (mod 2^64) is the exact sum of the low parts (< 2^47), so
// C = T 2^16 + R and C >= 2^63 exactly when T + (R >> 16) >= 2^47.
constexpr int kWrapParticles = 1 << 16;

// The particle ranges of a tile's workgroup: logical particle q lies in range r when cum[r] <= q < cum[r + 1], at
// sorted index rb[r] + q - cum[r] (local to the box).
struct TileRanges {
  int rb[8], cum[9];
  int nr;
};

// Adds (corner weight >> shift) of every particle in the ranges to the tile's cells in acc (LDS).
__device__ __forceinline__ void deposit_pass(const TileRanges tr, int tot, LPC_GLOBAL const float* __restrict__ pos,
                                             int64_t n, double scale, int nm, int x0, int y0, int z0,
                                             unsigned long long* acc, int shift) {
  const int64_t period = static_cast<int64_t>(nm) << kFracBits;
  // kUnroll particles per thread per round: all their position loads are issued before any is used
  constexpr int kUnroll = 4;
  for (int q0 = threadIdx.x; q0 < tot; q0 += kUnroll * kNT) {
    // every load is issued unconditionally (a thread past the end reloads the last particle and skips it below), so
    // the 3 kUnroll loads go out together instead of one conditional group at a time
    float px[kUnroll][3];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int q = min(q0 + u * kNT, tot - 1);
      int off = tr.rb[0];
#pragma unroll
      for (int r = 1; r < 8; ++r)
        if (r < tr.nr && q >= tr.cum[r]) off = tr.rb[r] - tr.cum[r];
      const int64_t i = off + q;
#pragma unroll
      for (int d = 0; d < 3; ++d) px[u][d] = pos[d * n + i];
    }
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      if (q0 + u * kNT >= tot) continue;
      uint32_t c[3], f[3];
      if (!fixed_coord3(px[u], scale, period, c, f)) continue;  // cannot happen for a bucketed particle
      // corner offsets relative to the tile origin (periodic), in [0, kT*) when inside
      int lx[2], ly[2], lz[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        int cx = static_cast<int>(c[0]) + a, cy = static_cast<int>(c[1]) + a, cz = static_cast<int>(c[2]) + a;
        if (cx == nm) cx = 0;
        if (cy == nm) cy = 0;
        if (cz == nm) cz = 0;
        lx[a] = cx - x0;
        ly[a] = cy - y0;
        lz[a] = cz - z0;
      }
      const uint32_t wx[2] = {kOne - f[0], f[0]}, wy[2] = {kOne - f[1], f[1]}, wz[2] = {kOne - f[2], f[2]};
      // one predicate per corner (inside the tile and a non-zero weight) instead of nested per-axis branches: each
      // divergent branch costs the scalar unit an exec-mask save and restore
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        const bool in_x = static_cast<unsigned>(lx[a]) < static_cast<unsigned>(kTX);
#pragma unroll
        for (int bb = 0; bb < 2; ++bb) {
          const bool in_xy = in_x && static_cast<unsigned>(ly[bb]) < static_cast<unsigned>(kTY);
          const uint64_t wab = static_cast<uint64_t>(wx[a]) * wy[bb];  // <= 2^32
#pragma unroll
          for (int e2 = 0; e2 < 2; ++e2) {
            const uint64_t wt = mul_weight(wab, wz[e2]) >> shift;
            if (in_xy && static_cast<unsigned>(lz[e2]) < static_cast<unsigned>(kTZ) && wt != 0)
              __hip_atomic_fetch_add(&acc[(lx[a] * kTY + ly[bb]) * kTZ + lz[e2]],
                                     static_cast<unsigned long long>(wt), __ATOMIC_RELAXED,
                                     __HIP_MEMORY_SCOPE_WORKGROUP);
          }
        }
      }
    }
  }
}

// Zeroes the tile's counts with 16-byte LDS stores, fully unrolled (no loop control on the scalar unit).
__device__ __forceinline__ void clear_tile(unsigned long long* acc, int tid) {
  static_assert(kTileCells % (2 * kNT) == 0, "whole 16-byte rounds");
  ulonglong2* a2 = reinterpret_cast<ulonglong2*>(acc);
#pragma unroll
  for (int m = 0; m < kTileCells / (2 * kNT); ++m) a2[tid + m * kNT] = make_ulonglong2(0ull, 0ull);
}

// Writes cell (j, k) of the x-planes 0 .. wx - 1 of the tile from acc: the int64 counts (TO_D false) or the FP32
// contrast v mscale - 1 (TO_D true). cell is the cell's index in plane 0, plane the cells of one x-plane. Returns
// whether a count has bit 63 set. Full-width tiles run the unrolled loop with no per-plane test.
template <bool TO_D>
__device__ __forceinline__ bool write_tile_column(const unsigned long long* acc, int tid, int wx, size_t cell,
                                                  size_t plane, LPC_GLOBAL unsigned long long* C, LPC_GLOBAL float* D,
                                                  double mscale) {
  bool overflow = false;
  auto put = [&](int i, size_t at) {
    const unsigned long long v = acc[i * kNT + tid];
    overflow |= (v >> 63) != 0;
    if constexpr (TO_D) {  // v in FP64 (hi 2^32 + lo, rounded once: the correctly rounded conversion), then C mscale - 1
      const double cv = fma(static_cast<double>(static_cast<uint32_t>(v >> 32)), 4294967296.0,
                            static_cast<double>(static_cast<uint32_t>(v)));
      D[at] = static_cast<float>(cv * mscale - 1.0);
    } else {
      C[at] = v;
    }
  };
  if (wx == kTX) {
#pragma unroll
    for (int i = 0; i < kTX; ++i, cell += plane) put(i, cell);
  } else {
    for (int i = 0; i < wx; ++i, cell += plane) put(i, cell);
  }
  return overflow;
}

__global__ __launch_bounds__(kNT) void k_deposit_tiles(const DepJob* __restrict__ jobs, const int* __restrict__ offs,
                                                       int njob, int total, const int* __restrict__ start,
                                                       int* __restrict__ flags) {
  __shared__ __align__(16) unsigned long long acc[kTileCells];
  const int w = blockIdx.x;
  if (w >= total) return;
  const int jb = __builtin_amdgcn_readfirstlane(find_job(to_const(offs), njob, w));
  const LPC_CONST DepJob& J = to_const(jobs)[jb];
  const int ntx = J.ntx, nty = J.nty, ntz = J.ntz, nm = J.nm;
  // neighbouring tiles (which share the particles of their boundary buckets) run on the same XCD
  // tiles in XCD-contiguous chunks of 64 (at 768^3: 0.748 ms with eighths of the tiles per XCD, 0.736 ms with chunks
  // of 32, 0.70 ms with 64; 48, 72, 96, 128 and 256 measured 0.71-0.75 ms)
  const int t = xcd_chunk_remap(w - offs[jb], offs[jb + 1] - offs[jb], 64);
  if (t >= ntx * nty * ntz) return;  // padding item
  const int tid = threadIdx.x;
  clear_tile(acc, tid);
  // t = (tx nty + ty) ntz + tz, split with the job's reciprocals instead of runtime divisions (exact: t < ntx nty ntz
  // and ntx (nty ntz)^2 < 2^32 for every mesh up to 1024)
  const int txy = static_cast<int>(fast_div(t, J.inv_z));  // tx nty + ty
  const int tx = static_cast<int>(fast_div(t, J.inv_yz));
  const int ty = txy - tx * nty, tz = t - txy * ntz;
  const int x0 = tx * kTX, y0 = ty * kTY, z0 = tz * kTZ;
  // the particle ranges (local indices, uniform): own tile, then the boundary bucket of each distinct lower
  // neighbour. All sixteen bucket bounds are loaded before any is used (one memory round trip, not eight).
  const int pbase = static_cast<int>(J.pbase);  // sort positions are int
  // an axis with one tile has no distinct lower neighbour
  const bool mx = ntx > 1, my = nty > 1, mz = ntz > 1;
  int bs[8], es[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int dx = (q >> 2) & 1, dy = (q >> 1) & 1, dz = q & 1;  // 1 = the lower neighbour along that axis
    const bool use = (mx || !dx) && (my || !dy) && (mz || !dz);
    const int sx = dx ? (tx == 0 ? ntx - 1 : tx - 1) : tx, sy = dy ? (ty == 0 ? nty - 1 : ty - 1) : ty,
              sz = dz ? (tz == 0 ? ntz - 1 : tz - 1) : tz;
    // always in range (an axis with one tile names the tile itself), so loaded without a branch; unused ones are
    // skipped below
    const int g = J.tbase + 2 * ((sx * nty + sy) * ntz + sz);
    (void)use;
    bs[q] = start[q == 0 ? g : g + 1];
    es[q] = start[g + 2];
  }
  int rb[8], cum[9];
  int nr = 0;
  cum[0] = 0;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int dx = (q >> 2) & 1, dy = (q >> 1) & 1, dz = q & 1;
    if ((mx || !dx) && (my || !dy) && (mz || !dz)) {
      const int b = __builtin_amdgcn_readfirstlane(bs[q] - pbase);
      const int e = __builtin_amdgcn_readfirstlane(es[q] - pbase);
      rb[nr] = b;
      cum[nr + 1] = cum[nr] + (e - b);
      ++nr;
    }
  }
  const int tot = cum[nr];
  // the ranges as uniform values (unused slots never selected: their start lies past tot)
  TileRanges tr;
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    tr.rb[r] = (r < nr) ? rb[r] : 0;
    tr.cum[r] = (r < nr) ? cum[r] : tot;
  }
  tr.cum[8] = tot;
  tr.nr = nr;
  __syncthreads();
  LPC_GLOBAL const float* pos = to_global(J.pos);
  deposit_pass(tr, tot, pos, J.n, J.scale, nm, x0, y0, z0, acc, 0);
  __syncthreads();
  // write the tile (cells outside the mesh on a narrow last tile are skipped): the exact int64 counts, and/or the
  // FP32 density contrast C mscale - 1 that the forward transform takes
  LPC_GLOBAL unsigned long long* C = to_global(reinterpret_cast<unsigned long long*>(J.dens));
  LPC_GLOBAL float* D = to_global(J.delta);
  const double mscale = J.mscale;
  const int wx_ = min(kTX, nm - x0), wy_ = min(kTY, nm - y0), wz_ = min(kTZ, nm - z0);
  bool overflow = false;
  // kNT = kTY kTZ threads: thread (j, k) writes its cell of every x-plane i, stepping one plane (nm^2 cells) at a
  // time; a wave's store covers two whole 128-byte rows
  static_assert(kNT == kTY * kTZ, "one thread per (y, z) cell of a tile plane");
  const int j = tid / kTZ, k = tid % kTZ;
  if (j < wy_ && k < wz_) {
    const size_t plane = static_cast<size_t>(nm) * nm;
    const size_t cell = (static_cast<size_t>(x0) * nm + (y0 + j)) * nm + (z0 + k);
    // (a job writes the contrast or the counts, not both; both pointers set would write both)
    if (D) overflow |= write_tile_column<true>(acc, tid, wx_, cell, plane, C, D, mscale);
    if (C) overflow |= write_tile_column<false>(acc, tid, wx_, cell, plane, C, D, mscale);
  }
  if (tot >= kWrapParticles) {  // uniform; rare (a tile reached by 65536 particles or more)
    unsigned long long S[kTX];
#pragma unroll
    for (int i = 0; i < kTX; ++i) S[i] = acc[i * kNT + tid];
    __syncthreads();
    clear_tile(acc, tid);
    __syncthreads();
    deposit_pass(tr, tot, pos, J.n, J.scale, nm, x0, y0, z0, acc, kFracBits);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kTX; ++i) {
      const unsigned long long T = acc[i * kNT + tid];
      const unsigned long long R = S[i] - (T << kFracBits);
      overflow |= (T + (R >> kFracBits)) >= (1ull << 47);
    }
  }
  if (overflow) atomicOr(flags + kFlagOverflow, 1);
}

// Copy sorted positions and momenta back to the caller's order.
__global__ __launch_bounds__(kNT) void k_unsort(const UnsortJob* __restrict__ jobs, const int* __restrict__ offs,
                                                int njob, int total) {
  for (int w = blockIdx.x; w < total; w += gridDim.x) {
    const int jb = __builtin_amdgcn_readfirstlane(find_job(to_const(offs), njob, w));
    const LPC_CONST UnsortJob& J = to_const(jobs)[jb];
    const int64_t n = J.n;
    const int64_t i = static_cast<int64_t>(xcd_remap(w - offs[jb], offs[jb + 1] - offs[jb])) * kNT + threadIdx.x;
    if (i >= n) continue;
    const int64_t o = to_global(J.orig)[i];
    LPC_GLOBAL const float* sp = to_global(J.spos);
    LPC_GLOBAL const float* sv = to_global(J.svel);
    LPC_GLOBAL float* p = to_global(J.pos);
    LPC_GLOBAL float* v = to_global(J.vel);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      p[d * n + o] = sp[d * n + i];
      v[d * n + o] = sv[d * n + i];
    }
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

// Lightcone test of one workgroup's particles (Sec. 6.1, 6.2): xs = wrapped positions at a_i, xe = unwrapped
// positions at a_{i+1}, v = momentum after the kick (the one at a_{i+1/2}), p1 / p2 = 2LPT displacements, ok = the
// thread holds a particle. Called by every thread of the workgroup (it has barriers).
//  1. Culling on the workgroup's bounding boxes (the rule of Sec. 6.2.3 applied to a tile of sorted particles
//     rather than to a whole replicate): an image can hold a crossing only if its start box comes within R_L(a_i)
//     of the observer and its end box reaches beyond R_L(a_{i+1}); the others are skipped.
//  2. Each particle tests each kept image: R_p,i <= R_L,i and R_p,i+1 > R_L,i+1; the crossing time comes from the
//     linear interpolation of R_p and R_L, the position from the drift to a_L (partial-drift table), the velocity is
//     the momentum at a_{i+1/2} (plus the frame momentum there for COLA). Records are appended with one counter atomic
//     per wave and image.
struct LcShared {
  float bb[kNT / 64][12];
  int list[kLcList];
  int nlist;
};

__device__ void lightcone_test(const LightconeStep& lc, const KickDrift& kd, float box, bool ok, const float xs[3],
                               const float xe[3], const float v[3], const float p1[3], const float p2[3], int index,
                               LcShared& sm) {
  const int tid = threadIdx.x, lane = __lane_id(), wave = tid / 64;
  const float inf = __builtin_inff();
  float b[12];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    b[d] = ok ? xs[d] : inf;
    b[3 + d] = ok ? xs[d] : -inf;
    b[6 + d] = ok ? xe[d] : inf;
    b[9 + d] = ok ? xe[d] : -inf;
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      b[d] = fminf(b[d], __shfl_xor(b[d], off));
      b[3 + d] = fmaxf(b[3 + d], __shfl_xor(b[3 + d], off));
      b[6 + d] = fminf(b[6 + d], __shfl_xor(b[6 + d], off));
      b[9 + d] = fmaxf(b[9 + d], __shfl_xor(b[9 + d], off));
    }
  }
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < 12; ++k) sm.bb[wave][k] = b[k];
  }
  if (tid == 0) sm.nlist = 0;
  __syncthreads();
#pragma unroll
  for (int k = 0; k < 12; ++k) {
    float m = sm.bb[0][k];
#pragma unroll
    for (int wv = 1; wv < kNT / 64; ++wv) m = (k % 6 < 3) ? fminf(m, sm.bb[wv][k]) : fmaxf(m, sm.bb[wv][k]);
    b[k] = m;
  }
  const float o[3] = {lc.ox, lc.oy, lc.oz};
  const float rli2 = lc.rli * lc.rli, rln2 = lc.rln * lc.rln;
  const int* __restrict__ reps = lc.reps;
  for (int r = tid; r < lc.nrep; r += kNT) {
    float dmin2 = 0.f, dmax2 = 0.f;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const float off = static_cast<float>(reps[4 * r + d]) * box;
      const float c = fmaxf(0.f, fmaxf(b[d] + off - o[d], o[d] - (b[3 + d] + off)));
      const float f = fmaxf(fabsf(b[6 + d] + off - o[d]), fabsf(b[9 + d] + off - o[d]));
      dmin2 += c * c;
      dmax2 += f * f;
    }
    if (dmin2 <= rli2 && dmax2 > rln2) {
      const int slot = atomicAdd(&sm.nlist, 1);
      if (slot < kLcList) sm.list[slot] = r;
    }
  }
  __syncthreads();
  const int nl = sm.nlist;
  const bool all = nl > kLcList;  // uniform
  const int count = all ? lc.nrep : nl;
  const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  for (int e = 0; e < count; ++e) {
    const int r = __builtin_amdgcn_readfirstlane(all ? e : sm.list[e]);
    float off[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) off[d] = static_cast<float>(reps[4 * r + d]) * box;
    float ri2 = 0.f, rn2 = 0.f;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const float ds = xs[d] + off[d] - o[d], de = xe[d] + off[d] - o[d];
      ri2 += ds * ds;
      rn2 += de * de;
    }
    const bool hit = ok && ri2 <= rli2 && rn2 > rln2;
    const unsigned long long mask = __ballot(hit);
    if (mask == 0ull) continue;
    unsigned long long base = 0;
    const int leader = __ffsll(static_cast<long long>(mask)) - 1;
    if (lane == leader) base = atomicAdd(lc.count, static_cast<unsigned long long>(__popcll(mask)));
    base = __shfl(base, leader);
    if (!hit) continue;
    const unsigned long long slot = base + __popcll(mask & below);
    if (slot >= static_cast<unsigned long long>(lc.capacity)) continue;
    const float rpi = sqrtf(ri2), rpn = sqrtf(rn2);
    float t = (lc.rli - rpi) / ((rpn - rpi) - (lc.rln - lc.rli));
    t = fminf(fmaxf(t, 0.f), 1.f);
    const float u = t * static_cast<float>(kLcTab - 1);
    const int k = min(static_cast<int>(u), kLcTab - 2);
    const float fr = u - static_cast<float>(k);
    const float* __restrict__ tb = lc.tab + 3 * k;
    const float q = tb[0] + fr * (tb[3] - tb[0]);
    const float e1 = tb[1] + fr * (tb[4] - tb[1]);
    const float e2 = tb[2] + fr * (tb[5] - tb[2]);
    LcRecord* rec = lc.out + slot;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      float xl = xs[d] + off[d] + q * v[d];
      float vl = v[d];
      if (kd.cola) {
        xl += e1 * p1[d] + e2 * p2[d];
        vl += lc.f1h * p1[d] + lc.f2h * p2[d];
      }
      rec->pos[d] = xl;
      rec->vel[d] = vl;
    }
    rec->a = lc.ai + t * (lc.aip1 - lc.ai);
    rec->index = index;
    rec->replicate = reps[4 * r + 3];
    rec->reserved = 0;
  }
  __syncthreads();  // sm is reused by the next item
}

template <bool LC>
__global__ __launch_bounds__(kNT) void k_gather_kick_drift(const PartJob* __restrict__ jobs,
                                                           const int* __restrict__ offs, int njob, int total,
                                                           KickDrift kd, LightconeStep lc, int* __restrict__ flags,
                                                           int* __restrict__ cnt, int* __restrict__ key,
                                                           int* __restrict__ rank) {
  __shared__ int sh[3 * kRankSlots];  // block_rank, when key != NULL
  for (int w = blockIdx.x; w < total; w += gridDim.x) {
    const int jb = __builtin_amdgcn_readfirstlane(find_job(to_const(offs), njob, w));
    const LPC_CONST PartJob& J = to_const(jobs)[jb];
    const int64_t n = J.n;
    const int64_t i = static_cast<int64_t>(w - offs[jb]) * kNT + threadIdx.x;
    const bool active = i < n;
    float x[3] = {0.f, 0.f, 0.f};
    // the lightcone's view of the drift: start, unwrapped end, momentum, displacements
    float xs[3] = {0.f, 0.f, 0.f}, xe[3] = {0.f, 0.f, 0.f}, vv[3] = {0.f, 0.f, 0.f};
    float q1[3] = {0.f, 0.f, 0.f}, q2[3] = {0.f, 0.f, 0.f};
    bool lc_ok = false;
    if (active) {
      LPC_GLOBAL float* pos = to_global(J.pos);
      LPC_GLOBAL float* vel = to_global(J.vel);
      LPC_GLOBAL const float* psi1 = to_global(J.psi1);
      LPC_GLOBAL const float* psi2 = to_global(J.psi2);
      x[0] = pos[i];
      x[1] = pos[n + i];
      x[2] = pos[2 * n + i];
      // the momentum and displacements are loaded with the position, so that their latency overlaps the gather's
      float v0[3], p1v[3] = {0.f, 0.f, 0.f}, p2v[3] = {0.f, 0.f, 0.f};
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        v0[d] = vel[d * n + i];
        if (kd.cola) {
          p1v[d] = psi1[d * n + i];
          p2v[d] = psi2[d * n + i];
        }
      }
      float g[3];
      if (!cic_gather(to_global(J.force), J.nm, J.scale, x[0], x[1], x[2], g)) {
        atomicOr(flags + kFlagNonfinite, 1);  // the particle is left as it is
      } else {
        const float box = J.box;
        lc_ok = true;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          float acc = g[d];
          const float p1 = p1v[d], p2 = p2v[d];
          if (kd.cola) acc += kd.d1 * p1 + kd.d2m * p2;
          const float v = v0[d] + kd.kick * acc;
          vel[d * n + i] = v;
          if (kd.do_drift) {
            float xn = x[d] + kd.drift * v;
            if (kd.cola) xn += kd.dd1 * p1 + kd.dd2 * p2;
            if constexpr (LC) {
              xs[d] = x[d];
              xe[d] = xn;
              vv[d] = v;
              q1[d] = p1;
              q2[d] = p2;
            }
            xn = wrap_box(xn, box);
            pos[d * n + i] = xn;
            x[d] = xn;
          }
        }
      }
    }
    if constexpr (LC) {
      __shared__ LcShared lsm;
      const int index = active ? (J.orig ? to_global(J.orig)[i] : static_cast<int>(i)) : -1;
      lightcone_test(lc, kd, J.box, lc_ok, xs, xe, vv, q1, q2, index, lsm);
    }
    if (key) {  // uniform: the next sort's key pass on the positions as stored (k_tile_key's arithmetic)
      int g = 0;
      if (active) {
        const int64_t period = static_cast<int64_t>(J.nm) << kFracBits;
        uint32_t c[3], f[3];
        bool ok = true;
#pragma unroll
        for (int d = 0; d < 3; ++d) ok &= fixed_coord(x[d], J.scale, period, &c[d], &f[d]);
        int b = 2 * J.ntx * J.nty * J.ntz;
        if (ok)
          b = bucket_of(c[0], c[1], c[2], J);
        else
          atomicOr(flags + kFlagNonfinite, 1);
        g = J.tbase + b;
      }
      const int r = block_rank(cnt, g, active, sh);
      if (active) {
        key[J.pbase + i] = g;
        rank[J.pbase + i] = r;
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
    const int64_t o = J.orig ? to_global(J.orig)[i] : i;  // output in the caller's order
    grad[o] = g[0];
    grad[n + o] = g[1];
    grad[2 * n + o] = g[2];
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

// One workgroup per item of kNT particles. (The kernels keep their grid-stride loops, so any grid is correct; a grid
// capped at 8192 workgroups left the last round of resident workgroups part-full: at 768^3 the scatter took 0.60
// against 0.53 ms and the gather/kick/drift 1.19 against 1.11 ms.)
unsigned grid_of(const WorkTable& wt) { return static_cast<unsigned>(wt.total); }

}  // namespace

hipError_t fill_i32(int* p, size_t count, int value, hipStream_t s) {
  if (count == 0) return hipSuccess;
  size_t blocks = (count + kNT - 1) / kNT;
  if (blocks > 65536) blocks = 65536;
  k_fill_i32<<<static_cast<unsigned>(blocks), kNT, 0, s>>>(p, count, value);
  return hipGetLastError();
}

hipError_t launch_tile_key(const SortJob* jobs, WorkTable wt, int* cnt, int* key, int* rank, int* flags,
                           hipStream_t s) {
  if (wt.total <= 0) return hipSuccess;
  k_tile_key<<<grid_of(wt), kNT, 0, s>>>(jobs, wt.offs, wt.njob, wt.total, cnt, key, rank, flags);
  return hipGetLastError();
}

int scan_blocks(int count) { return (count + kScanBlock - 1) / kScanBlock; }

hipError_t launch_scan(const int* cnt, int* start, int count, int* block_sums, hipStream_t s) {
  const int nb = scan_blocks(count);
  if (nb == 0) return hipErrorInvalidValue;
  k_scan_local<<<nb, kNT, 0, s>>>(cnt, start, count, block_sums);
  k_scan_sums<<<1, kNT, 0, s>>>(block_sums, nb, start, count);
  k_scan_add<<<nb, kNT, 0, s>>>(start, count, block_sums);
  return hipGetLastError();
}

hipError_t launch_scatter(const SortJob* jobs, WorkTable wt, const int* key, const int* rank, const int* start,
                          hipStream_t s) {
  if (wt.total <= 0) return hipSuccess;
  k_scatter<<<grid_of(wt), kNT, 0, s>>>(jobs, wt.offs, wt.njob, wt.total, key, rank, start);
  return hipGetLastError();
}

hipError_t launch_deposit_tiles(const DepJob* jobs, WorkTable wt, const int* start, int* flags, hipStream_t s) {
  if (wt.total <= 0) return hipSuccess;
  k_deposit_tiles<<<static_cast<unsigned>(wt.total), kNT, 0, s>>>(jobs, wt.offs, wt.njob, wt.total, start, flags);
  return hipGetLastError();
}

hipError_t launch_unsort(const UnsortJob* jobs, WorkTable wt, hipStream_t s) {
  if (wt.total <= 0) return hipSuccess;
  k_unsort<<<grid_of(wt), kNT, 0, s>>>(jobs, wt.offs, wt.njob, wt.total);
  return hipGetLastError();
}

hipError_t launch_gather_kick_drift(const PartJob* jobs, WorkTable wt, KickDrift kd, int* flags, int* cnt, int* key,
                                    int* rank, hipStream_t s) {
  if (wt.total <= 0) return hipSuccess;
  if (key && (!cnt || !rank)) return hipErrorInvalidValue;
  k_gather_kick_drift<false><<<grid_of(wt), kNT, 0, s>>>(jobs, wt.offs, wt.njob, wt.total, kd,
                                                                        LightconeStep{}, flags, cnt, key, rank);
  return hipGetLastError();
}

hipError_t launch_gather_kick_drift_lc(const PartJob* jobs, WorkTable wt, KickDrift kd, const LightconeStep& lc,
                                       int* flags, int* cnt, int* key, int* rank, hipStream_t s) {
  if (wt.total <= 0) return hipSuccess;
  if ((key && (!cnt || !rank)) || !kd.do_drift || !lc.tab || (lc.nrep > 0 && !lc.reps) || !lc.count ||
      (lc.capacity > 0 && !lc.out))
    return hipErrorInvalidValue;
  k_gather_kick_drift<true><<<grid_of(wt), kNT, 0, s>>>(jobs, wt.offs, wt.njob, wt.total, kd, lc, flags,
                                                                       cnt, key, rank);
  return hipGetLastError();
}

hipError_t launch_gather(const PartJob* jobs, WorkTable wt, int* flags, hipStream_t s) {
  if (wt.total <= 0) return hipSuccess;
  k_gather<<<grid_of(wt), kNT, 0, s>>>(jobs, wt.offs, wt.njob, wt.total, flags);
  return hipGetLastError();
}

hipError_t launch_frame(const PartJob* jobs, WorkTable wt, float f1, float f2, hipStream_t s) {
  if (wt.total <= 0) return hipSuccess;
  k_frame_velocity<<<grid_of(wt), kNT, 0, s>>>(jobs, wt.offs, wt.njob, wt.total, f1, f2);
  return hipGetLastError();
}

}  // namespace kern
}  // namespace lpc
