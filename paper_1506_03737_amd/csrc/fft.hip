// 3-D real FFTs of liblpc as three LDS-staged passes over HBM (Sec. 2.4 steps 2-3 of Howlett, Manera & Percival
// 2015: forward FFT of the density, Poisson solve and gradient in k-space, inverse FFT per force component).
//
// Layout: a real mesh is x-major float[n][n][n]; its half spectrum is float2[n][n][pitch] with kz = 0..n/2 used
// (pitch = n/2 + 1 rounded up to 8 complex values, 64 bytes, so every row starts on a 64-byte boundary).
// Forward: z pass (r2c of each row via a length-n/2 complex FFT and the even/odd split), y pass, x pass.
// Inverse: x pass, y pass, z pass (c2r via the same split). The force path fuses the forward x pass, the Poisson /
// deconvolution multiply and the inverse x transforms into one kernel, so the density spectrum is read once and never
// written back; it stores the x gradient and the potential, whose y and z gradients the y and z passes apply.
//
// Every kernel is batched: workgroup w takes item w of a work table of (job, tile) items, where a job is one mesh of
// one box, so one launch per pass serves any number of boxes of uneven sizes (see WorkTable). (A persistent
// grid-stride loop over the items measured slower: it raised register pressure past the four-waves-per-SIMD limit.)
#include <hip/hip_runtime.h>

#include <algorithm>
#include <utility>
#include <cmath>

#include "fft_device.h"

namespace lpc {
namespace kern {

// p[s], pmask[s] and tw_off[s] of a plan whose radices are set
static void set_strides(Plan1D* p);

bool make_plan(int n, Plan1D* p, bool radix12) {
  if (n < 1) return false;
  int m = n, ns = 0;
  int odd[kMaxStages];
  for (int r : {5, 3}) {
    while (m % r == 0) {
      if (ns >= kMaxStages) return false;
      odd[ns++] = r;
      m /= r;
    }
  }
  int k = 0;
  while (m % 2 == 0) {
    m /= 2;
    ++k;
  }
  if (m != 1) return false;
  // powers of two: radix-8 stages, the remainder as one radix-4 or radix-2 stage (8 x 2 becomes 4 x 4)
  int pow2[kMaxStages], np = 0;
  int n8 = k / 3, rem = k % 3;
  if (rem == 1 && n8 > 0) {
    --n8;
    pow2[np++] = 4;
    pow2[np++] = 4;
    rem = 0;
  }
  for (int i = 0; i < n8; ++i) pow2[np++] = 8;
  if (rem == 1) pow2[np++] = 2;
  if (rem == 2) pow2[np++] = 4;
  // a radix-4 and a radix-3 stage merge into one radix-12 stage (one LDS round trip fewer)
  int i4 = -1, i3 = -1;
  for (int i = 0; i < np; ++i)
    if (pow2[i] == 4) i4 = i;
  for (int i = 0; i < ns; ++i)
    if (odd[i] == 3) i3 = i;
  const bool r12 = radix12 && i4 >= 0 && i3 >= 0;
  if (ns + np - (r12 ? 1 : 0) > kMaxStages) return false;
  p->n = n;
  p->nst = 0;
  for (int i = 0; i < np; ++i)
    if (!(r12 && i == i4)) p->radix[p->nst++] = pow2[i];
  if (r12) p->radix[p->nst++] = 12;
  for (int i = 0; i < ns; ++i)
    if (!(r12 && i == i3)) p->radix[p->nst++] = odd[i];
  set_strides(p);
  return true;
}

Plan1D reversed_plan(const Plan1D& p) {
  Plan1D r = p;
  for (int s = 0; s < p.nst; ++s) r.radix[s] = p.radix[p.nst - 1 - s];
  set_strides(&r);
  return r;
}

static void set_strides(Plan1D* p) {
  int prod = 1, off = 0;
  for (int s = 0; s < p->nst; ++s) {
    p->p[s] = prod;
    p->pmask[s] = ((prod & (prod - 1)) == 0) ? prod - 1 : -1;
    p->tw_off[s] = off;
    off += prod * (p->radix[s] - 1);
    prod *= p->radix[s];
  }
}

int mesh_pitch(int n) { return ((n / 2 + 1) + 7) / 8 * 8; }

namespace {

// Lets the kernel take up to 160 KB of dynamic LDS. If the attribute cannot be set, a launch that asks for more than
// the default fails, and the launcher reports it through hipGetLastError.
template <class K>
void allow_big_lds(K kernel) {
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                            160 * 1024);
}

// The transforms of the workloads' meshes (768 for the single box and the learned form's fine run, 192 / 256 / 320 for
// the batched form and the coarse run) with compile-time plans when the job's plan is one of them and the tile can
// hold it, fft_tile otherwise; both compute the same stages with the same twiddle table. HALF selects the plans of the
// half-length z transforms, otherwise those of the full-length x and y transforms; a kernel carries only its own kind.
template <class F, class PL>
__device__ __forceinline__ bool try_fixed(float2* tile, const float2* tw, const PL& pl, int tid) {
  if (!F::matches(pl)) return false;
  F::run(tile, tw, tid);
  return true;
}

template <bool INV, int EPT, int B, int BP, bool HALF, bool R12 = true, class PL>
__device__ __forceinline__ void fft_tile_fast(float2* tile, const float2* tw, const PL& pl, int tid) {
  // full-length plans (make_plan): 768 = 8 x 8 x 12, 320 = 8 x 8 x 5, 256 = 8 x 8 x 4, 192 = 8 x 8 x 3;
  // half-length with radix 12: 384 = 4 x 8 x 12, 160 = 8 x 4 x 5, 128 = 4 x 4 x 8, 96 = 8 x 12;
  // half-length without radix 12: 384 = 4 x 4 x 8 x 3, 160, 128 as above, 96 = 8 x 4 x 3
  if constexpr (!HALF) {
    if (try_fixed<FixedFFT<INV, EPT, B, BP, 8, 8, 12>>(tile, tw, pl, tid)) return;
    if (try_fixed<FixedFFT<INV, EPT, B, BP, 8, 8, 5>>(tile, tw, pl, tid)) return;
    if (try_fixed<FixedFFT<INV, EPT, B, BP, 8, 8, 4>>(tile, tw, pl, tid)) return;
    if (try_fixed<FixedFFT<INV, EPT, B, BP, 8, 8, 3>>(tile, tw, pl, tid)) return;
  } else {
    if constexpr (R12) {
      if (try_fixed<FixedFFT<INV, EPT, B, BP, 4, 8, 12>>(tile, tw, pl, tid)) return;
      if (try_fixed<FixedFFT<INV, EPT, B, BP, 8, 12>>(tile, tw, pl, tid)) return;
    } else {
      if (try_fixed<FixedFFT<INV, EPT, B, BP, 4, 4, 8, 3>>(tile, tw, pl, tid)) return;
      if (try_fixed<FixedFFT<INV, EPT, B, BP, 8, 4, 3>>(tile, tw, pl, tid)) return;
    }
    if (try_fixed<FixedFFT<INV, EPT, B, BP, 8, 4, 5>>(tile, tw, pl, tid)) return;
    if (try_fixed<FixedFFT<INV, EPT, B, BP, 4, 4, 8>>(tile, tw, pl, tid)) return;
  }
  fft_tile<INV, EPT, R12>(tile, tw, pl, B, BP, tid);
}

// fft_tile_fast with the tile's fill and drain folded into the first and last stages: with GIN the input comes from
// load(row, col) (the tile is not filled first; mid() runs while the first loads are in flight), with GOUT the
// output goes to store(row, col, value). Full-length transforms; plans other than the compiled ones fill the tile,
// run fft_tile and store from it. The twiddles in tw must be in LDS by the first barrier (mid() may write them).
template <class F, class PL, bool GIN, bool GOUT, bool PAIRS, class Load, class Pair, class Mid, class Store>
__device__ __forceinline__ bool try_fixed_io(float2* tile, const float2* tw, const PL& pl, int tid, Load load,
                                             Pair pair, Mid mid, Store store) {
  if (!F::matches(pl)) return false;
  F::template run_io<GIN, GOUT, PAIRS>(tile, tw, tid, load, pair, mid, store);
  return true;
}

// PAIRS: tile column b < B / 2 is pair(row, x) and column b + B / 2 is x itself, for x = load(row, b) of a B / 2
// column source (load takes source columns only). Columns transform independently, so for a column that store skips
// (past the mesh edge) load may return any finite value: the kernels reload the item's last column there instead of
// predicating the load and clearing its register.
template <bool INV, int EPT, int B, int BP, bool GIN, bool GOUT, bool PAIRS = false, class PL, class Load, class Pair,
          class Mid, class Store>
__device__ __forceinline__ void fft_io_fast(float2* tile, const float2* tw, const PL& pl, int tid, Load load, Pair pair,
                                            Mid mid, Store store) {
#define LPC_TRY_IO(...)                                                                                          \
  if (try_fixed_io<FixedFFT<INV, EPT, B, BP, __VA_ARGS__>, PL, GIN, GOUT, PAIRS>(tile, tw, pl, tid, load, pair, mid, \
                                                                             store))                             \
    return;
  LPC_TRY_IO(8, 8, 12)
  LPC_TRY_IO(12, 8, 8)    // 768 in the force's y passes
  LPC_TRY_IO(8, 8, 5)
  LPC_TRY_IO(8, 8, 4)
  LPC_TRY_IO(8, 8, 3)
  LPC_TRY_IO(4, 4, 8, 8)  // 1024: the large box
  LPC_TRY_IO(4, 8, 12)    // 384: the learned form's fine training runs
#undef LPC_TRY_IO
  // other plans: fill the tile (n B <= EPT kFftNT values), transform it in place, store it. With 12 or more points per
  // thread (the largest meshes) the loads go out in unrolled batches of four per thread, so that each batch's loads
  // are in flight together; the 80-register instances keep a plain loop (the batches would spill them).
  const int n = pl.n, count = n * B;
  if constexpr (GIN && EPT < 12) {
    for (int e = tid; e < count; e += kFftNT) {
      const int j = e / B, b = e % B;
      if constexpr (PAIRS) {
        const float2 x = load(j, b % (B / 2));
        tile[j * BP + b] = (b < B / 2) ? pair(j, x) : x;
      } else {
        tile[j * BP + b] = load(j, b);
      }
    }
    mid();
    __syncthreads();
  } else if constexpr (GIN) {
    constexpr int H = 4, NH = (EPT + H - 1) / H;
#pragma unroll
    for (int half = 0; half < NH; ++half) {
      float2 v[H];
#pragma unroll
      for (int m = 0; m < H; ++m) {
        const int e = tid + (half * H + m) * kFftNT;
        v[m] = make_float2(0.f, 0.f);
        if (e < count) {
          const int j = e / B, b = e % B;
          if constexpr (PAIRS) {
            const float2 x = load(j, b % (B / 2));
            v[m] = (b < B / 2) ? pair(j, x) : x;
          } else {
            v[m] = load(j, b);
          }
        }
      }
      if (half == 0) mid();
#pragma unroll
      for (int m = 0; m < H; ++m) {
        const int e = tid + (half * H + m) * kFftNT;
        if (e < count) tile[(e / B) * BP + (e % B)] = v[m];
      }
    }
    __syncthreads();
  }
  fft_tile<INV, EPT, true>(tile, tw, pl, B, BP, tid);
  if constexpr (GOUT) {
#pragma unroll
    for (int m = 0; m < EPT; ++m) {
      const int e = tid + m * kFftNT;
      if (e < count) store(e / B, e % B, tile[(e / B) * BP + (e % B)]);
    }
  }
}

// Job of work item w: the last j with offs[j] <= w (binary search; offs is uniform, so scalar loads).
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

// ---------------------------------------------------------------------------------------------------------------
// Every kernel stages its global loads through registers in fully unrolled batches before writing the LDS tile: a
// runtime-bounded load loop would wait out the HBM latency once per element.

// z pass, forward r2c. An item transforms B consecutive rows of n reals. Each row is read as h = n/2 complex values
// z[m] = x[2m] + i x[2m+1]; after the length-h FFT, X[k] = E[k] + exp(-2 pi i k / n) O[k] with
// E[k] = (Z[k] + conj Z[h-k]) / 2 and O[k] = (Z[k] - conj Z[h-k]) / (2 i), for k = 0..h.
template <bool FIXED, int B, int EPT>
__global__ __launch_bounds__(kFftNT, 4) void k_fft_z_r2c(const ZR2CJob* __restrict__ jobs,
                                                         const int* __restrict__ offs, int njob, int total,
                                                         int* __restrict__ flags) {
  constexpr int BP = B + 1;
  extern __shared__ float2 smem[];
  {
    const int w = blockIdx.x;
    const int tid = threadIdx.x;
    if (w >= total) return;
    const int jb = __builtin_amdgcn_readfirstlane(find_job(to_const(offs), njob, w));
    const LPC_CONST ZR2CJob& J = to_const(jobs)[jb];
    const int n = J.n, h = n / 2, nrows = J.nrows;
    // each XCD takes a contiguous range of row blocks (r2c 0.72 -> 0.68 ms, c2r 2.25 -> 2.20 ms at 768^3)
    const int row0 = xcd_remap(w - offs[jb], offs[jb + 1] - offs[jb]) * B;
    if (row0 >= nrows) return;  // padding item (uniform; no LDS touched)
    float2* tile = smem;
    float2* tw = tile + h * BP;
    float2* roots = tw + h;
    const int count = h * B;
    // Element e = tid + m kFftNT of the tile is (row b, point j) = divmod(e, h): one division per thread, then steps
    // of kFftNT = dq h + dr.
    const int dq = kFftNT / h, dr = kFftNT - dq * h;
    const int b0 = tid / h, j0 = tid - b0 * h;
    // The item's rows are contiguous in the input, so element e is at offset row0 h + e (in complex values); rows past
    // the last are not read.
    const int valid = min(count, (nrows - row0) * h);
    // the tables' loads go out first, so that writing them to LDS waits for them only
    const TableRegs<float2> r_tw = table_load(J.tw, h, tid), r_roots = table_load(J.roots, h + 1, tid);
    if (FIXED) {
      LPC_GLOBAL const ulonglong2* in =
          reinterpret_cast<LPC_GLOBAL const ulonglong2*>(to_global(static_cast<const uint64_t*>(J.in))) +
          static_cast<size_t>(row0) * h;
      constexpr int H = EPT / 2;
      int bb = b0, jj = j0;
#pragma unroll 1
      for (int half = 0; half < 2; ++half) {
        ulonglong2 raw[H];
        int b = bb, j = jj;
#pragma unroll
        for (int m = 0; m < H; ++m) {
          const int e = tid + (half * H + m) * kFftNT;
          raw[m] = make_ulonglong2(0ull, 0ull);
          if (e < valid) raw[m] = in[e];
        }
        if (half == 0) {
          table_store(tw, r_tw, h, tid);
          table_store(roots, r_roots, h + 1, tid);
        }
        bool overflow = false;
        b = bb;
        j = jj;
#pragma unroll
        for (int m = 0; m < H; ++m) {
          const int e = tid + (half * H + m) * kFftNT;
          if (e < count) {
            overflow |= ((raw[m].x | raw[m].y) >> 63) != 0;
            float2 v = make_float2(0.f, 0.f);
            if (row0 + b < nrows) {
              v.x = static_cast<float>(static_cast<double>(raw[m].x) * J.mscale - 1.0);
              v.y = static_cast<float>(static_cast<double>(raw[m].y) * J.mscale - 1.0);
            }
            tile[j * BP + b] = v;
          }
          b += dq;
          j += dr;
          if (j >= h) {
            j -= h;
            ++b;
          }
        }
        bb = b;
        jj = j;
        if (overflow) atomicOr(flags + kFlagOverflow, 1);
      }
    } else {
      LPC_GLOBAL const float2* in = to_global(static_cast<const float2*>(J.in)) + static_cast<size_t>(row0) * h;
      float2 v[EPT];
#pragma unroll
      for (int m = 0; m < EPT; ++m) {
        const int e = tid + m * kFftNT;
        v[m] = make_float2(0.f, 0.f);
        if (e < valid) v[m] = in[e];
      }
      table_store(tw, r_tw, h, tid);
      table_store(roots, r_roots, h + 1, tid);
      int b = b0, j = j0;
#pragma unroll
      for (int m = 0; m < EPT; ++m) {
        const int e = tid + m * kFftNT;
        if (e < count) tile[j * BP + b] = v[m];
        b += dq;
        j += dr;
        if (j >= h) {
          j -= h;
          ++b;
        }
      }
    }
    __syncthreads();
    fft_tile_fast<false, EPT, B, BP, true>(tile, tw, J.pl, tid);
    LPC_GLOBAL float2* out = to_global(J.out);
    const int pitch = J.pitch;
    // Output in pairs (k, h - k), k <= h / 2, of each row: with E = (Z[k] + conj Z[h-k]) / 2,
    // O = (Z[k] - conj Z[h-k]) / (2 i) and t = exp(-2 pi i k / n) O, X[k] = E + t and X[h-k] = conj(E - t)
    // (Z[h] = Z[0]). Unit u = (row b, pair k) = divmod(u, h / 2 + 1): one division per thread, then steps.
    const int hk = h / 2 + 1, npair = B * hk;
    const int dqp = kFftNT / hk, drp = kFftNT - dqp * hk;
    int b = tid / hk, k = tid - (tid / hk) * hk;
    for (int u = tid; u < npair; u += kFftNT) {
      const int row = row0 + b;
      if (row < nrows) {
        const float2 zk = tile[k * BP + b];
        const float2 zm = tile[(k == 0 ? 0 : h - k) * BP + b];
        const float2 E = cscale(cadd(zk, cconj(zm)), 0.5f);
        const float2 O = cscale(rot<false>(csub(zk, cconj(zm))), 0.5f);  // (zk - conj zm) / (2 i)
        const float2 t = cmul(roots[k], O);
        LPC_GLOBAL float2* o = out + static_cast<size_t>(row) * pitch;
        o[k] = cadd(E, t);
        if (2 * k != h) o[h - k] = cconj(csub(E, t));
      }
      b += dqp;
      k += drp;
      if (k >= hk) {
        k -= hk;
        ++b;
      }
    }
  }
}

// Load/store of a strided tile of B columns: element (j, b) <-> ptr[j * astr + b], for b < bw, with n B <= EPT kFftNT.
// Loads go out in two unrolled batches of EPT / 2 per thread (enough bytes in flight per CU to cover HBM latency at
// a register cost that keeps four waves per SIMD): strided_issue loads batch `half` into registers, strided_put
// writes it to the tile, so a kernel can do other work (its twiddle tables) while the first batch is in flight.
template <int B, int H>
__device__ __forceinline__ void strided_issue(float2 (&v)[H], LPC_GLOBAL const float2* __restrict__ ptr, int64_t astr,
                                              int n, int bw, int tid, int half) {
  const int count = n * B;
#pragma unroll
  for (int m = 0; m < H; ++m) {
    const int e = tid + (half * H + m) * kFftNT;
    const int j = e / B, b = e % B;
    v[m] = make_float2(0.f, 0.f);
    if (e < count && b < bw) v[m] = ptr[j * astr + b];
  }
}

template <int B, int H>
__device__ __forceinline__ void strided_put(float2* tile, const float2 (&v)[H], int n, int tid, int half) {
  constexpr int BP = strided_pitch(B);
  const int count = n * B;
#pragma unroll
  for (int m = 0; m < H; ++m) {
    const int e = tid + (half * H + m) * kFftNT;
    if (e < count) tile[(e / B) * BP + (e % B)] = v[m];
  }
}

template <int B, int EPT = kEPT>
__device__ __forceinline__ void store_strided(const float2* tile, LPC_GLOBAL float2* __restrict__ ptr, int64_t astr, int n,
                                              int bw, int tid) {
  constexpr int BP = strided_pitch(B);
  const int count = n * B;
#pragma unroll
  for (int m = 0; m < EPT; ++m) {
    const int e = tid + m * kFftNT;
    const int j = e / B, b = e % B;
    if (e < count && b < bw) ptr[j * astr + b] = tile[j * BP + b];
  }
}

// ---------------------------------------------------------------------------------------------------------------
// Strided complex pass (in place). A tile is B consecutive columns (contiguous in memory) x n points along the
// axis. Within a component, tiles are XCD-remapped so that neighbouring tiles (which share cache lines at their
// edges) run on the same XCD. Each thread owns at most EPT points of its column (n B <= EPT kFftNT); with EPT <= 8
// the kernel fits in 80 VGPRs (three workgroups of 8 waves per CU where the LDS tile allows it); larger EPT gets
// 128 (a cap of 96 would also give two workgroups per CU, and spills).
template <bool INV, int B, int EPT>
__global__ __launch_bounds__(kFftNT, (EPT <= 8) ? 6 : 4) void k_fft_axis(const AxisJob* __restrict__ jobs,
                                                        const int* __restrict__ offs, int njob, int total) {
  extern __shared__ float2 smem[];
  {
    const int w = blockIdx.x;
    const int tid = threadIdx.x;
    if (w >= total) return;
    const int jb = __builtin_amdgcn_readfirstlane(find_job(to_const(offs), njob, w));
    const LPC_CONST AxisJob& J = to_const(jobs)[jb];
    const int local = w - offs[jb];
    const int comp = local / J.per_comp;
    // XCD-contiguous chunks of 32 items rather than eighths (forward y 0.785 -> 0.759 ms at 768^3; the other strided
    // passes and the z passes measured no better that way)
    const int t = xcd_chunk_remap(local - comp * J.per_comp, J.per_comp, 32);
    const int outer = t / J.ntc, ct = t - outer * J.ntc;
    const int n = J.n;
    if (outer >= n) return;  // padding item
    const int c0 = ct * B, bw = min(B, J.ncols - c0);
    float2* tile = smem;
    float2* tw = smem + n * strided_pitch(B);
    LPC_GLOBAL float2* ptr = to_global(J.base + comp * J.cstr + outer * J.ostr + c0);
    const uint32_t astr = static_cast<uint32_t>(J.astr);  // j astr < 2^32 for every mesh up to 1024
    // the first stage reads the columns from HBM and the last writes them back: the tile holds only the stages between
    const TableRegs<float2> twr = table_load(J.tw, n, tid);
    auto load = [&](int j, int b) { return ptr[static_cast<uint32_t>(j) * astr + min(b, bw - 1)]; };
    auto mid = [&]() { table_store(tw, twr, n, tid); };
    auto store = [&](int j, int b, float2 v) {
      if (b < bw) ptr[static_cast<uint32_t>(j) * astr + b] = v;
    };
    auto none = [](int, float2 x) { return x; };
    fft_io_fast<INV, EPT, B, strided_pitch(B), true, true>(tile, tw, J.pl, tid, load, none, mid, store);
  }
}

// ---------------------------------------------------------------------------------------------------------------
// Inverse y pass of the force. Items of component 0 transform a tile of B columns of A (the x gradient) in place.
// Items of component 1 take B / 2 columns of the x-transformed potential psi from C and stack them twice in their
// tile, as i k_y psi (columns b) and as psi (columns B / 2 + b): one B-column transform gives the y gradient, stored
// to B, and psi, stored back to C (k_z is constant along y; the z pass applies i k_z as it loads C). An item reads and
// writes only its own columns, so items do not race.
template <int B, int EPT>
__global__ __launch_bounds__(kFftNT, EPT <= 8 ? 6 : 4) void k_fft_y_grad(
    const YGradJob* __restrict__ jobs, const int* __restrict__ offs, int njob, int total) {
  constexpr int BP = strided_pitch(B), H = EPT / 2, BH = B / 2;
  extern __shared__ float2 smem[];
  const int w = blockIdx.x;
  const int tid = threadIdx.x;
  if (w >= total) return;
  const int jb = __builtin_amdgcn_readfirstlane(find_job(to_const(offs), njob, w));
  const LPC_CONST YGradJob& J = to_const(jobs)[jb];
  const int local = w - offs[jb];
  const int n = J.n;
  float2* tile = smem;
  float2* tw = smem + n * BP;
  const TableRegs<float2> twr = table_load(J.tw, n, tid);
  auto mid = [&]() { table_store(tw, twr, n, tid); };
  if (local < J.per_comp) {  // component 0 (uniform)
    const int t = xcd_remap(local, J.per_comp);
    const int outer = t / J.ntc, ct = t - outer * J.ntc;
    if (outer >= n) return;  // padding item
    const int c0 = ct * B, bw = min(B, J.ncols - c0);
    LPC_GLOBAL float2* ptr = to_global(J.A + static_cast<int64_t>(outer) * J.ostr + c0);
    const uint32_t astr = static_cast<uint32_t>(J.astr);
    auto load = [&](int j, int b) { return ptr[static_cast<uint32_t>(j) * astr + min(b, bw - 1)]; };
    auto store = [&](int j, int b, float2 v) {
      if (b < bw) ptr[static_cast<uint32_t>(j) * astr + b] = v;
    };
    auto none = [](int, float2 x) { return x; };
    fft_io_fast<true, EPT, B, BP, true, true>(tile, tw, J.pl, tid, load, none, mid, store);
    return;
  }
  const int t = xcd_remap(local - J.per_comp, J.per_comp1);
  const int outer = t / J.ntc1, ct = t - outer * J.ntc1;
  if (outer >= n) return;  // padding item
  const int c0 = ct * BH, bw = min(BH, J.ncols - c0);
  const int64_t off = static_cast<int64_t>(outer) * J.ostr + c0;
  LPC_GLOBAL const float2* src = to_global(J.C + off);
  LPC_GLOBAL float2* dB = to_global(J.B + off);
  LPC_GLOBAL float2* dC = to_global(J.C + off);
  const uint32_t astr = static_cast<uint32_t>(J.astr);
  const int half = n / 2;
  const float kf = J.kf;
  // tile column b < BH holds i k_y psi of psi's column b, column BH + b psi itself; they go to B and back to C.
  // Each psi value is loaded once and feeds both columns.
  auto load = [&](int j, int bh) { return src[static_cast<uint32_t>(j) * astr + min(bh, bw - 1)]; };
  auto iky = [&](int j, float2 v) {
    const float ky = (j == half) ? 0.f : kf * static_cast<float>(j <= half ? j : j - n);
    return make_float2(-ky * v.y, ky * v.x);
  };
  auto store = [&](int j, int b, float2 v) {
    const int bh = b % BH;
    if (bh < bw) (b < BH ? dB : dC)[static_cast<uint32_t>(j) * astr + bh] = v;
  };
  fft_io_fast<true, EPT, B, BP, true, true, true>(tile, tw, J.pl, tid, load, iky, mid, store);
}

// ---------------------------------------------------------------------------------------------------------------
// A compile-time plan (radices Rs in order, or reversed with REV): stage s has radix r(s), sub-transform length p(s)
// and its twiddles at off(s) of the plan's table (the layout make_plan gives it).
template <bool REV, int... Rs>
struct ChainPlan {
  static constexpr int K = sizeof...(Rs);
  static constexpr int N = (Rs * ...);
  static constexpr int fwd[K] = {Rs...};
  static constexpr int r(int s) { return REV ? fwd[K - 1 - s] : fwd[s]; }
  static constexpr int p(int s) {
    int q = 1;
    for (int t = 0; t < s; ++t) q *= r(t);
    return q;
  }
  static constexpr int off(int s) {
    int o = 0;
    for (int t = 0; t < s; ++t) o += p(t) * (r(t) - 1);
    return o;
  }
};

// Stages 1 .. K - 2 of plan CP in the tile.
template <class CP, bool INV, int EPT, int B, int BP, int... S>
__device__ __forceinline__ void chain_mid_stages(float2* tile, const float2* tw, int tid,
                                                 std::integer_sequence<int, S...>) {
  (fft_stage_c<CP::r(S + 1), INV, EPT, CP::N, CP::p(S + 1), B, BP>(tile, tw + CP::off(S + 1), tid), ...);
}

// The fused x pass on 8-column tiles with its three transforms chained through registers, for the plans 8 x 8 x R
// (R = 12, 5, 4, 3: meshes 768, 320, 256, 192) and 4 x 4 x 8 x 8 (1024). The forward transform's last stage (radix
// RL) leaves each thread's MB butterflies in its registers: thread (i, b) = (tid / 8, tid % 8) holds rows
// i + m 64 + r N / RL of column b, in natural order (MB = 1 for 8 x 8 x R, 2 for 1024). factor(row, g, ph) turns each
// into psi_hat (ph) and i k_x psi_hat (g) there. Both inverse transforms run the plan in reverse order, whose first
// stage (radix RL) takes exactly those rows, so neither spectrum goes back through the tile between the transforms:
// for 768, 12 LDS passes and 9 barriers per tile instead of 18 and 15. The reversed plan's twiddles wait in registers
// (r_twr) and replace the forward ones in LDS once the forward transform has read them, so one table's worth of LDS
// serves both (at 1024 that lets two workgroups share a CU).
template <int M, int... Rs, class PL, class Load, class Mid, class MakeFactor, class StoreA, class StoreC>
__device__ __forceinline__ bool x_poisson_chained(float2* tile, float2* tw, const TableRegs<float2>& r_twr,
                                                  const PL& pl, int tid, Load load, Mid mid, MakeFactor make_factor,
                                                  StoreA store_a, StoreC store_c) {
  constexpr int B = 8, BP = strided_pitch(B);
  using Fwd = FixedFFT<false, M, B, BP, Rs...>;
  if constexpr (!Fwd::kFits) {
    return false;
  } else {
    if (!Fwd::matches(pl)) return false;
    using F = ChainPlan<false, Rs...>;
    using V = ChainPlan<true, Rs...>;
    constexpr int N = F::N, K = F::K, RF = F::r(0), RL = F::r(K - 1);
    constexpr int MB = (N / RL) * B / kFftNT;
    static_assert(MB * kFftNT == (N / RL) * B, "the last stage's butterflies split evenly over the threads");
    using Mids = std::make_integer_sequence<int, K - 2>;
    // forward: the first stage from HBM, the middle stages in the tile, the last into registers
    fft_stage_from_global<RF, false, M, N, B, BP>(tile, load, mid, tid);
    __syncthreads();
    chain_mid_stages<F, false, M, B, BP>(tile, tw, tid, Mids{});
    float2 g[MB][RL], ph[MB][RL];
    fft_stage_to_regs<RL, false, N, F::p(K - 1), B, BP, MB>(tile, tw + F::off(K - 1), tid, g);
    {
      const auto factor = make_factor();
      const int i0 = tid / B;
#pragma unroll
      for (int m = 0; m < MB; ++m) {
#pragma unroll
        for (int r = 0; r < RL; ++r) factor(i0 + m * (kFftNT / B) + r * (N / RL), g[m][r], ph[m][r]);
      }
    }
    __syncthreads();  // the tile and the forward twiddles have been read
    table_store(tw, r_twr, N, tid);
    // first inverse: i k_x psi_hat -> the x gradient in A
    fft_stage_from_regs<RL, true, N, B, BP, MB>(tile, g, tid);
    __syncthreads();
    chain_mid_stages<V, true, M, B, BP>(tile, tw, tid, Mids{});
    fft_stage_to_global<RF, true, M, N, V::p(K - 1), B, BP>(tile, tw + V::off(K - 1), store_a, tid);
    __syncthreads();
    // second inverse: psi_hat -> the x-transformed potential in C
    fft_stage_from_regs<RL, true, N, B, BP, MB>(tile, ph, tid);
    __syncthreads();
    chain_mid_stages<V, true, M, B, BP>(tile, tw, tid, Mids{});
    fft_stage_to_global<RF, true, M, N, V::p(K - 1), B, BP>(tile, tw + V::off(K - 1), store_c, tid);
    return true;
  }
}

// Fused x pass of the force. With psi_hat = -delta_hat / (k^2 W^p Nm^3) (zero at k = 0; W = prod_d sinc^2(pi n_d /
// Nm); the 1/Nm^3 of the inverse transform folded in), the gradient spectra are g_hat_j = i k_j psi_hat, zero on the
// Nyquist plane of axis j. Along the x transform k_y and k_z are constant (per tile and per column), so
//   IFFT_x(g_hat_x) = IFFT_x(i k_x psi_hat) -> A,   IFFT_x(g_hat_{y,z}) = i k_{y,z} IFFT_x(psi_hat), IFFT_x(psi_hat) -> C:
// one forward and two inverse transforms per tile, two spectra written. psi_hat is kept between them. The CHAIN
// instances (B = 8, M <= 12) run every job's transforms chained through registers (x_poisson_chained): the host
// launches them only when every job's plan is 8 x 8 x R (poisson_chainable). Otherwise each thread owns the points of
// column b at rows j0 + m S, at most M of them (M = n B / kFftNT rounded up to 8, 12 or 16): with M <= 12 they stay
// in the thread's registers, so the workgroup needs one LDS tile and two workgroups fit on a CU; with M = 16 a second
// LDS tile holds them (the registers would spill). The two forms are separate instances because the generic form's
// register allocation would otherwise cover the chained form's too (and spill). The chained M = 8 instance (the
// 192-320 meshes) is capped at 80 VGPRs, so that three workgroups fit on a CU (48-box step 30.86 -> 30.25 ms).
template <int B, int M, bool CHAIN>
__global__ __launch_bounds__(kFftNT, (CHAIN && M <= 8) ? 6 : ((CHAIN || M <= 12) ? 4 : 2)) void k_fft_x_poisson(
    const PoissonJob* __restrict__ jobs, const int* __restrict__ offs, int njob, int total) {
  constexpr int BP = strided_pitch(B), S = kFftNT / B;
  constexpr bool kRegs = CHAIN || M <= 12;  // psi_hat in registers (else a second LDS tile)
  extern __shared__ float2 smem[];
  {
    const int w = blockIdx.x;
    const int tid = threadIdx.x;
    if (w >= total) return;
    const int jb = __builtin_amdgcn_readfirstlane(find_job(to_const(offs), njob, w));
    const LPC_CONST PoissonJob& J = to_const(jobs)[jb];
    const int n = J.nm, nm = J.nm, nh = nm / 2 + 1, pitch = J.pitch;
    const int t = xcd_remap(w - offs[jb], offs[jb + 1] - offs[jb]);
    const int y = t / J.ntc, ct = t - y * J.ntc;
    if (y >= n) return;  // padding item
    float2* tile = smem;
    float2* ph_lds = tile + n * BP;  // psi_hat when !kRegs
    float2* tw = tile + (kRegs ? 1 : 2) * n * BP;
    float* win = reinterpret_cast<float*>(tw + n);  // sinc^2(pi m / n), m <= n / 2 (even in m)
    const int c0 = ct * B, bw = min(B, nh - c0);
    const uint32_t astr = static_cast<uint32_t>(nm) * static_cast<uint32_t>(pitch);  // j astr < 2^32 (Nm <= 1024)
    const int64_t off = static_cast<int64_t>(y) * pitch + c0;
    LPC_GLOBAL float2* gA = to_global(J.A + off);
    LPC_GLOBAL float2* gC = to_global(J.C + off);
    const int half = nm / 2;
    const int ny = (y <= half) ? y : y - nm;
    const float kf = J.kf, inv_m3 = J.inv_m3;
    const int deconv = J.deconv;
    // The Poisson factor of this thread's column b = tid % B (read once the window table is in LDS):
    // factor(j, g, ph) takes the forward spectrum at row j in g and leaves psi_hat in ph and i k_x psi_hat in g.
    auto make_factor = [&]() {
      const int b = tid % B, nz = c0 + b;
      const bool col_ok = b < bw;
      const float wyz = win[min(y, n - y)] * win[min(nz, half)];
      const int nyz2 = ny * ny + nz * nz;
      return [=](int j, float2& g, float2& ph) {
        const int nx = (j <= half) ? j : j - nm;
        const float k2 = kf * kf * static_cast<float>(nx * nx + nyz2);
        float sc = 0.f;
        if (k2 > 0.f && col_ok) {
          const float W = win[min(j, n - j)] * wyz;
          const float wp = (deconv == 0) ? 1.f : (deconv == 1 ? W : W * W);
          sc = -inv_m3 * __builtin_amdgcn_rcpf(k2 * wp);  // hardware reciprocal (1 ulp) instead of a division
        }
        ph = make_float2(sc * g.x, sc * g.y);
        const float kx = (nx == half) ? 0.f : kf * static_cast<float>(nx);
        g = make_float2(-kx * ph.y, kx * ph.x);
      };
    };
    auto load = [&](int j, int b) { return gA[static_cast<uint32_t>(j) * astr + min(b, bw - 1)]; };
    auto store_a = [&](int j, int b, float2 v) {
      if (b < bw) gA[static_cast<uint32_t>(j) * astr + b] = v;
    };
    auto store_c = [&](int j, int b, float2 v) {
      if (b < bw) gC[static_cast<uint32_t>(j) * astr + b] = v;
    };
    if constexpr (CHAIN) {
      static_assert(B == 8, "the chained form takes 8-column tiles");
      // the tables' loads go out first; mid() writes the forward twiddles and the window to LDS while the first
      // stage's loads are in flight, the reversed plan's twiddles stay in registers until the forward pass is done
      const TableRegs<float2> r_tw = table_load(J.tw, n, tid), r_twr = table_load(J.tw_rev, n, tid);
      const TableRegs<float> r_win = table_load(J.win, n / 2 + 1, tid);
      auto mid = [&]() {
        table_store(tw, r_tw, n, tid);
        table_store(win, r_win, n / 2 + 1, tid);
      };
#define LPC_CHAIN(...) \
  if (x_poisson_chained<M, __VA_ARGS__>(tile, tw, r_twr, J.pl, tid, load, mid, make_factor, store_a, store_c)) return;
      LPC_CHAIN(8, 8, 12)
      LPC_CHAIN(8, 8, 5)
      LPC_CHAIN(8, 8, 4)
      LPC_CHAIN(8, 8, 3)
      LPC_CHAIN(4, 4, 8, 8)
#undef LPC_CHAIN
      return;
    } else {
      auto none = [](int, float2 x) { return x; };
      auto nothing = []() {};
      auto no_load = [](int, int) { return make_float2(0.f, 0.f); };
      auto no_store = [](int, int, float2) {};
      {
        // forward transform: the first stage reads delta_hat from HBM; the tables are copied while its loads are in
        // flight; the result stays in the tile (natural order)
        const TableRegs<float2> r_tw = table_load(J.tw, n, tid);
        const TableRegs<float> r_win = table_load(J.win, n / 2 + 1, tid);
        auto mid = [&]() {
          table_store(tw, r_tw, n, tid);
          table_store(win, r_win, n / 2 + 1, tid);
        };
        fft_io_fast<false, M, B, BP, true, false>(tile, tw, J.pl, tid, load, none, mid, no_store);
      }

      // Each thread touches only its own points between the barriers that bracket the inverse transforms.
      float2 ph[kRegs ? M : 1];
      {
        const auto factor = make_factor();
        const int b = tid % B, j0 = tid / B;
#pragma unroll
        for (int m = 0; m < M; ++m) {
          const int j = j0 + m * S;
          if (j >= n) continue;
          float2 g = tile[j * BP + b], psi;
          factor(j, g, psi);
          if (kRegs)
            ph[kRegs ? m : 0] = psi;
          else
            ph_lds[j * BP + b] = psi;
          tile[j * BP + b] = g;  // i k_x psi_hat
        }
      }
      __syncthreads();
      // first inverse transform: the last stage writes the x gradient to A
      fft_io_fast<true, M, B, BP, false, true>(tile, tw, J.pl, tid, no_load, none, nothing, store_a);
      __syncthreads();
      {
        // (the empty asm keeps the comp-invariant indices of the first inverse transform from staying live)
        int ltid = tid;
        asm volatile("" : "+v"(ltid));
        const int b = ltid % B, j0 = ltid / B;
#pragma unroll
        for (int m = 0; m < M; ++m) {
          const int j = j0 + m * S;
          if (j < n) tile[j * BP + b] = kRegs ? ph[kRegs ? m : 0] : ph_lds[j * BP + b];
        }
        __syncthreads();
        // the x-transformed potential: the y and z gradients are i k_y and i k_z times it (applied by the y and z
        // passes); the last stage writes it to C
        fft_io_fast<true, M, B, BP, false, true>(tile, tw, J.pl, ltid, no_load, none, nothing, store_c);
      }
    }
  }
}

// ---------------------------------------------------------------------------------------------------------------
// z pass, inverse c2r. An item transforms R rows of each of NC spectra; tile column r NC + c holds spectrum c of
// row r (B = NC R columns). With X the half spectrum of a real row,
//   Z[k] = (X[k] + conj X[h-k]) + i exp(+2 pi i k / n) (X[k] - conj X[h-k]),  h = n/2, k < h,
// and the unnormalised length-h inverse FFT of Z gives x[2m] + i x[2m+1]. Output rows are NC-interleaved.
// Each thread owns at most EPT points of a column (h <= EPT S); with EPT <= 12 the kernel fits in 80 VGPRs, so
// LDS-light tiles run three workgroups per CU.
template <int NC, int R, int EPT>
__global__ __launch_bounds__(kFftNT, (EPT <= 12) ? 6 : 4) void k_fft_z_c2r(const ZC2RJob* __restrict__ jobs,
                                                         const int* __restrict__ offs, int njob, int total) {
  constexpr int B = NC * R, BP = B + 1;
  extern __shared__ float2 smem[];
  {
    const int w = blockIdx.x;
    const int tid = threadIdx.x;
    if (w >= total) return;
    const int jb = __builtin_amdgcn_readfirstlane(find_job(to_const(offs), njob, w));
    const LPC_CONST ZC2RJob& J = to_const(jobs)[jb];
    const int n = J.n, h = n / 2, nrows = J.nrows, pitch = J.pitch;
    const int row0 = xcd_remap(w - offs[jb], offs[jb + 1] - offs[jb]) * R;  // as in the r2c: XCD-contiguous rows
    if (row0 >= nrows) return;  // padding item
    float2* tile = smem;                 // (h + 1) x BP
    float2* tw = tile + (h + 1) * BP;    // stage twiddles (h)
    float2* roots = tw + h;              // exp(-2 pi i k / n), k <= h
    LPC_GLOBAL const float2* in0 = to_global(J.in0);
    LPC_GLOBAL const float2* in1 = to_global(J.in1);
    LPC_GLOBAL const float2* in2 = to_global(J.in2);
    const float kz3 = J.kz3;
    // Loads, spectrum by spectrum: element e = tid + m kFftNT of a spectrum's R rows below the Nyquist point is
    // (row r, frequency k) = divmod(e, h), the same for every spectrum, so the offsets are stepped once (one division
    // per thread, then steps of kFftNT = dq h + dr) and each spectrum's base pointer is a compile-time choice. R h <=
    // B h / NC <= EPT kFftNT / NC, so MC loads per thread and spectrum cover it. The R NC Nyquist points (k = h) are
    // one load each for the first R NC threads. Tile column of (row r, spectrum c): r NC + c.
    constexpr int MC = (EPT + NC - 1) / NC;
    const int per = R * h;
    const int dq = kFftNT / h, dr = kFftNT - dq * h;
    // the tables' loads go out first, so that writing them to LDS waits for them only
    const TableRegs<float2> r_tw = table_load(J.tw, h, tid), r_roots = table_load(J.roots, h + 1, tid);
    {
      int64_t goff[MC];  // global element offset (row0 + r) pitch + k, or -1 for no element
      int loff[MC];      // tile offset k BP + r NC
      int kk[MC];
      {
        int r = tid / h, k = tid - (tid / h) * h;
#pragma unroll
        for (int m = 0; m < MC; ++m) {
          const bool ok = tid + m * kFftNT < per && row0 + r < nrows;
          goff[m] = ok ? static_cast<int64_t>(row0 + r) * pitch + k : -1;
          loff[m] = k * BP + r * NC;
          kk[m] = k;
          r += dq;
          k += dr;
          if (k >= h) {
            k -= h;
            ++r;
          }
        }
      }
      float2 v[NC][MC];
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        LPC_GLOBAL const float2* src = (c == 0) ? in0 : (c == 1 ? in1 : in2);
#pragma unroll
        for (int m = 0; m < MC; ++m) {
          v[c][m] = make_float2(0.f, 0.f);
          if (goff[m] >= 0) v[c][m] = src[goff[m]];
        }
      }
      const int nyq_r = tid / NC, nyq_c = tid - nyq_r * NC;  // Nyquist point of tile column tid
      float2 nyq = make_float2(0.f, 0.f);
      if (tid < B && row0 + nyq_r < nrows) {
        LPC_GLOBAL const float2* src = (nyq_c == 0) ? in0 : (nyq_c == 1 ? in1 : in2);
        nyq = src[static_cast<size_t>(row0 + nyq_r) * pitch + h];
      }
      // the tables are written while the loads are in flight
      table_store(tw, r_tw, h, tid);
      table_store(roots, r_roots, h + 1, tid);
#pragma unroll
      for (int c = 0; c < NC; ++c) {
#pragma unroll
        for (int m = 0; m < MC; ++m) {
          if (tid + m * kFftNT < per) {
            float2 x = v[c][m];
            // the third spectrum is psi: i k_z psi (applied here, once every load is issued)
            if (NC == 3 && c == 2 && kz3 != 0.f) {
              const float kz = kz3 * static_cast<float>(kk[m]);
              x = make_float2(-kz * x.y, kz * x.x);
            }
            tile[loff[m] + c] = x;
          }
        }
      }
      // i k_z psi is zero on the Nyquist plane
      if (tid < B) tile[h * BP + tid] = (NC == 3 && nyq_c == 2 && kz3 != 0.f) ? make_float2(0.f, 0.f) : nyq;
    }
    __syncthreads();
    {
      const int hk = h / 2 + 1;
      const int dqk = kFftNT / hk, drk = kFftNT - dqk * hk;
      int col = tid / hk, k = tid - (tid / hk) * hk;
      for (int e = tid; e < hk * B; e += kFftNT) {
        const float2 xk = tile[k * BP + col];
        const float2 xm = tile[(h - k) * BP + col];
        const float2 t = roots[k];
        // Z[k] = (xk + conj xm) + i conj(t) (xk - conj xm) = S + u, and
        // Z[h-k] = (xm + conj xk) - i t (xm - conj xk) = conj(S - u)
        const float2 S = cadd(xk, cconj(xm));
        const float2 u = rot<true>(cmulc(csub(xk, cconj(xm)), t));
        if (k != 0 && 2 * k != h) tile[(h - k) * BP + col] = cconj(csub(S, u));
        tile[k * BP + col] = cadd(S, u);
        col += dqk;
        k += drk;
        if (k >= hk) {
          k -= hk;
          ++col;
        }
      }
    }
    __syncthreads();
    fft_tile_fast<true, EPT, B, BP, true, NC != 3>(tile, tw, J.pl, tid);  // NC = 3: plans without radix 12
    // Output: tile row m of row r holds points 2m and 2m + 1 of every spectrum (columns r NC .. r NC + NC - 1),
    // i.e. 2 NC consecutive floats of the NC-interleaved output row. One (row, m) unit per thread: NC 8-byte LDS
    // reads at a stride of BP float2 between lanes (conflict-free for odd BP) and NC 8-byte stores, contiguous across
    // lanes.
    const int rowlen = NC * n, hm = n / 2;
    const float scale = J.scale;
    const int units = min(R, nrows - row0) * hm;
    LPC_GLOBAL float* dst = to_global(J.out) + static_cast<size_t>(row0) * rowlen;
    // (the empty asm keeps the store loop's per-thread indices from being computed before the transform)
    int stid = tid;
    asm volatile("" : "+v"(stid));
    if ((reinterpret_cast<uintptr_t>(J.out) & 7) == 0) {
      // unit u = r hm + m: one division per thread, then steps of kFftNT = dqs hm + drs
      const int dqs = kFftNT / hm, drs = kFftNT - dqs * hm;
      int r = stid / hm, m = stid - r * hm;
#pragma unroll 1
      for (int u = stid; u < units; u += kFftNT) {
        const float2* src = tile + m * BP + r * NC;
        LPC_GLOBAL float2* o = reinterpret_cast<LPC_GLOBAL float2*>(dst + static_cast<size_t>(r) * rowlen + 2 * NC * m);
        if (NC == 3) {
          const float2 a = src[0], b = src[1], c = src[2];
          o[0] = make_float2(a.x * scale, b.x * scale);
          o[1] = make_float2(c.x * scale, a.y * scale);
          o[2] = make_float2(b.y * scale, c.y * scale);
        } else {
          const float2 a = src[0];
          o[0] = make_float2(a.x * scale, a.y * scale);
        }
        r += dqs;
        m += drs;
        if (m >= hm) {
          m -= hm;
          ++r;
        }
      }
    } else {
      for (int f = stid; f < units * 2 * NC; f += kFftNT) {
        const int r = f / rowlen, q = f - r * rowlen;
        const int jj = q / NC, c = q - jj * NC;
        const float2 z = tile[(jj >> 1) * BP + r * NC + c];
        dst[f] = ((jj & 1) ? z.y : z.x) * scale;
      }
    }
  }
}

struct Init {
  Init() {
    allow_big_lds(k_fft_z_r2c<true, 8, 8>);
    allow_big_lds(k_fft_z_r2c<true, 8, 12>);
    allow_big_lds(k_fft_z_r2c<true, 8, 16>);
    allow_big_lds(k_fft_z_r2c<true, 16, 8>);
    allow_big_lds(k_fft_z_r2c<true, 16, 12>);
    allow_big_lds(k_fft_z_r2c<true, 16, 16>);
    allow_big_lds(k_fft_z_r2c<true, 32, 8>);
    allow_big_lds(k_fft_z_r2c<true, 32, 12>);
    allow_big_lds(k_fft_z_r2c<true, 32, 16>);
    allow_big_lds(k_fft_z_r2c<false, 8, 8>);
    allow_big_lds(k_fft_z_r2c<false, 8, 12>);
    allow_big_lds(k_fft_z_r2c<false, 8, 16>);
    allow_big_lds(k_fft_z_r2c<false, 16, 8>);
    allow_big_lds(k_fft_z_r2c<false, 16, 12>);
    allow_big_lds(k_fft_z_r2c<false, 16, 16>);
    allow_big_lds(k_fft_z_r2c<false, 32, 8>);
    allow_big_lds(k_fft_z_r2c<false, 32, 12>);
    allow_big_lds(k_fft_z_r2c<false, 32, 16>);
    allow_big_lds(k_fft_axis<true, 8, 8>);
    allow_big_lds(k_fft_axis<true, 8, 12>);
    allow_big_lds(k_fft_axis<true, 8, 16>);
    allow_big_lds(k_fft_axis<true, 16, 8>);
    allow_big_lds(k_fft_axis<true, 16, 12>);
    allow_big_lds(k_fft_axis<true, 16, 16>);
    allow_big_lds(k_fft_axis<true, 32, 8>);
    allow_big_lds(k_fft_axis<true, 32, 12>);
    allow_big_lds(k_fft_axis<true, 32, 16>);
    allow_big_lds(k_fft_axis<false, 8, 8>);
    allow_big_lds(k_fft_axis<false, 8, 12>);
    allow_big_lds(k_fft_axis<false, 8, 16>);
    allow_big_lds(k_fft_axis<false, 16, 8>);
    allow_big_lds(k_fft_axis<false, 16, 12>);
    allow_big_lds(k_fft_axis<false, 16, 16>);
    allow_big_lds(k_fft_axis<false, 32, 8>);
    allow_big_lds(k_fft_axis<false, 32, 12>);
    allow_big_lds(k_fft_axis<false, 32, 16>);
    allow_big_lds(k_fft_y_grad<8, 8>);
    allow_big_lds(k_fft_y_grad<8, 12>);
    allow_big_lds(k_fft_y_grad<8, 16>);
    allow_big_lds(k_fft_y_grad<16, 8>);
    allow_big_lds(k_fft_y_grad<16, 12>);
    allow_big_lds(k_fft_y_grad<16, 16>);
    allow_big_lds(k_fft_y_grad<32, 8>);
    allow_big_lds(k_fft_y_grad<32, 12>);
    allow_big_lds(k_fft_y_grad<32, 16>);
    allow_big_lds(k_fft_x_poisson<8, 8, true>);
    allow_big_lds(k_fft_x_poisson<8, 12, true>);
    allow_big_lds(k_fft_x_poisson<8, 16, true>);
    allow_big_lds(k_fft_x_poisson<4, 8, false>);
    allow_big_lds(k_fft_x_poisson<8, 8, false>);
    allow_big_lds(k_fft_x_poisson<8, 12, false>);
    allow_big_lds(k_fft_x_poisson<8, 16, false>);
    allow_big_lds(k_fft_x_poisson<16, 8, false>);
    allow_big_lds(k_fft_x_poisson<16, 12, false>);
    allow_big_lds(k_fft_x_poisson<16, 16, false>);
    allow_big_lds(k_fft_z_c2r<1, 8, kEPT>);
    allow_big_lds(k_fft_z_c2r<1, 16, kEPT>);
    allow_big_lds(k_fft_z_c2r<1, 32, kEPT>);
    allow_big_lds(k_fft_z_c2r<3, 4, 8>);
    allow_big_lds(k_fft_z_c2r<3, 4, 12>);
    allow_big_lds(k_fft_z_c2r<3, 4, 16>);
    allow_big_lds(k_fft_z_c2r<3, 8, 8>);
    allow_big_lds(k_fft_z_c2r<3, 8, 12>);
    allow_big_lds(k_fft_z_c2r<3, 8, 16>);
    allow_big_lds(k_fft_z_c2r<3, 16, 8>);
    allow_big_lds(k_fft_z_c2r<3, 16, 12>);
    allow_big_lds(k_fft_z_c2r<3, 16, 16>);
  }
};

void ensure_init() { static Init once; }

// One workgroup per work item (the table's total is a multiple of 8, so blockIdx.x % 8 is the item's XCD slot).
unsigned item_grid(int total) { return total > 0 ? static_cast<unsigned>(total) : 0u; }


}  // namespace

size_t lds_z_r2c(int n, int B) { return sizeof(float2) * (static_cast<size_t>(n / 2) * (B + 1) + n / 2 + n / 2 + 1); }
size_t lds_axis(int n, int B) { return sizeof(float2) * (static_cast<size_t>(n) * strided_pitch(B) + n); }
// Points per thread of a strided tile of B columns at length n (n B / kFftNT), rounded up to 8, 12 or 16.
int axis_points(int n, int B) {
  const long pts = (static_cast<long>(n) * B + kFftNT - 1) / kFftNT;
  return pts <= 8 ? 8 : (pts <= 12 ? 12 : 16);
}

// Points per thread of a forward r2c z tile of B rows (B columns of length n / 2), rounded up to 8, 12 or 16.
int r2c_points(int n, int B) {
  const long pts = (static_cast<long>(n / 2) * B + kFftNT - 1) / kFftNT;
  return pts <= 8 ? 8 : (pts <= 12 ? 12 : 16);
}

// Points per thread of a three-spectrum c2r z tile of R rows (B = 3 R columns of length n / 2, S = kFftNT / B
// threads per column), rounded up to 8, 12 or 16 (the kernel's EPT).
int c2r_points(int n, int R) {
  const int S = kFftNT / (3 * R);
  const int pts = (n / 2 + S - 1) / S;
  return pts <= 8 ? 8 : (pts <= 12 ? 12 : 16);
}

// Points per thread of the fused x + Poisson tile, n B / kFftNT rounded up to 8, 12 or 16 (the kernel's M).
int poisson_points(int n, int B) {
  const long pts = (static_cast<long>(n) * B + kFftNT - 1) / kFftNT;
  return pts <= 8 ? 8 : (pts <= 12 ? 12 : 16);
}

bool poisson_chainable(const Plan1D& pl) {
  if (pl.nst == 4) return pl.radix[0] == 4 && pl.radix[1] == 4 && pl.radix[2] == 8 && pl.radix[3] == 8;
  if (pl.nst != 3 || pl.radix[0] != 8 || pl.radix[1] != 8) return false;
  const int r = pl.radix[2];
  return r == 12 || r == 5 || r == 4 || r == 3;
}

size_t lds_x_poisson(int n, int B, int M, bool chained) {
  const size_t tiles = (chained || M <= 12) ? 1 : 2;
  // tile(s), the stage twiddles (the chained form's two tables take turns), the window
  return sizeof(float2) * (tiles * static_cast<size_t>(n) * strided_pitch(B) + n) + sizeof(float) * (n / 2 + 1);
}
size_t lds_z_c2r(int n, int B) {
  return sizeof(float2) * (static_cast<size_t>(n / 2 + 1) * (B + 1) + n / 2 + n / 2 + 1);
}

// Columns of a strided tile: the most of 8, 16, 32 with n * B <= kTileElems (8 for n > 512).
int strided_cols(int n) { return (n <= 256) ? 32 : (n <= 512 ? 16 : 8); }

namespace {

// A z-pass tile of B interleaved columns (rows times spectra) at length n: the loads cover B (h + 1) values with
// kEPT + 1 per thread, and each of the S = kFftNT / B threads of a column takes at most kEPT points per stage.
bool rows_fit(int n, int B) {
  const long h = n / 2;
  return B >= 1 && B <= kFftNT && B * (h + 1) <= kTileElems + kFftNT &&
         h * B <= static_cast<long>(kEPT) * (kFftNT / B) * B;
}

// A strided tile of B columns at length n: n B values loaded with kEPT per thread, kEPT points per thread per stage.
bool cols_fit(int n, int B) {
  return B >= 1 && B <= kFftNT && static_cast<long>(n) * B <= static_cast<long>(kEPT) * (kFftNT / B) * B;
}

constexpr size_t kMaxLds = 160 * 1024;

}  // namespace

// Rows of a z-pass tile for NC interleaved spectra: the largest power of two up to 32 that fits (rows_fit).
int z_rows(int n, int nc) {
  int best = 1;
  for (int r = 1; r <= 32; r *= 2) {
    if (!rows_fit(n, nc * r)) break;
    best = r;
  }
  return best;
}

bool tile_ok(TileKind kind, int n, int w) {
  switch (kind) {
    case TileKind::kZRows:  // forward r2c and single-spectrum c2r z passes (instances 8, 16, 32)
      return (w == 8 || w == 16 || w == 32) && rows_fit(n, w) && lds_z_r2c(n, w) <= kMaxLds &&
             lds_z_c2r(n, w) <= kMaxLds;
    case TileKind::kAxisCols:  // strided y / x passes (instances 8, 16, 32)
      return (w == 8 || w == 16 || w == 32) && cols_fit(n, w) && lds_axis(n, w) <= kMaxLds;
    case TileKind::kPoissonCols:  // fused x + Poisson pass (instances 4, 8, 16)
      return (w == 4 || w == 8 || w == 16) && cols_fit(n, w) &&
             lds_x_poisson(n, w, poisson_points(n, w), false) <= kMaxLds;
    case TileKind::kForceC2RRows:  // three-component c2r z pass (instances 4, 8, 16)
      return (w == 4 || w == 8 || w == 16) && rows_fit(n, 3 * w) && lds_z_c2r(n, 3 * w) <= kMaxLds;
  }
  return false;
}

void init_kernels() { ensure_init(); }

hipError_t launch_z_r2c(const ZR2CJob* jobs, WorkTable wt, bool fixed, int B, int P, size_t lds, int* flags,
                        hipStream_t s) {
  ensure_init();
  const unsigned g = item_grid(wt.total);
  if (g == 0) return hipSuccess;
  if ((B != 8 && B != 16 && B != 32) || (P != 8 && P != 12 && P != 16)) return hipErrorInvalidValue;
#define LPC_ZR2C(F, BB, PP) k_fft_z_r2c<F, BB, PP><<<g, kFftNT, lds, s>>>(jobs, wt.offs, wt.njob, wt.total, flags)
#define LPC_ZR2C_P(F, BB) \
  if (P == 8) LPC_ZR2C(F, BB, 8); else if (P == 12) LPC_ZR2C(F, BB, 12); else LPC_ZR2C(F, BB, 16)
  if (fixed) {
    if (B == 8) { LPC_ZR2C_P(true, 8); } else if (B == 16) { LPC_ZR2C_P(true, 16); } else { LPC_ZR2C_P(true, 32); }
  } else {
    if (B == 8) { LPC_ZR2C_P(false, 8); } else if (B == 16) { LPC_ZR2C_P(false, 16); } else { LPC_ZR2C_P(false, 32); }
  }
#undef LPC_ZR2C_P
#undef LPC_ZR2C
  return hipGetLastError();
}

hipError_t launch_axis(const AxisJob* jobs, WorkTable wt, bool inverse, int B, int P, size_t lds, hipStream_t s) {
  ensure_init();
  const unsigned g = item_grid(wt.total);
  if (g == 0) return hipSuccess;
#define LPC_AXIS(INV, BB, PP) k_fft_axis<INV, BB, PP><<<g, kFftNT, lds, s>>>(jobs, wt.offs, wt.njob, wt.total)
#define LPC_AXIS_P(INV, BB) \
  if (P == 8) LPC_AXIS(INV, BB, 8); else if (P == 12) LPC_AXIS(INV, BB, 12); else if (P == 16) LPC_AXIS(INV, BB, 16); \
  else return hipErrorInvalidValue
  if (inverse) {
    if (B == 8) { LPC_AXIS_P(true, 8); } else if (B == 16) { LPC_AXIS_P(true, 16); } else if (B == 32) { LPC_AXIS_P(true, 32); }
    else return hipErrorInvalidValue;
  } else {
    if (B == 8) { LPC_AXIS_P(false, 8); } else if (B == 16) { LPC_AXIS_P(false, 16); } else if (B == 32) { LPC_AXIS_P(false, 32); }
    else return hipErrorInvalidValue;
  }
#undef LPC_AXIS_P
#undef LPC_AXIS
  return hipGetLastError();
}

hipError_t launch_y_grad(const YGradJob* jobs, WorkTable wt, int B, int P, size_t lds, hipStream_t s) {
  ensure_init();
  const unsigned g = item_grid(wt.total);
  if (g == 0) return hipSuccess;
#define LPC_YG(BB, PP) k_fft_y_grad<BB, PP><<<g, kFftNT, lds, s>>>(jobs, wt.offs, wt.njob, wt.total)
#define LPC_YG_P(BB) \
  if (P == 8) LPC_YG(BB, 8); else if (P == 12) LPC_YG(BB, 12); else if (P == 16) LPC_YG(BB, 16); \
  else return hipErrorInvalidValue
  if (B == 8) { LPC_YG_P(8); } else if (B == 16) { LPC_YG_P(16); } else if (B == 32) { LPC_YG_P(32); }
  else return hipErrorInvalidValue;
#undef LPC_YG_P
#undef LPC_YG
  return hipGetLastError();
}

hipError_t launch_poisson(const PoissonJob* jobs, WorkTable wt, int B, int M, bool chained, size_t lds, hipStream_t s) {
  ensure_init();
  const unsigned g = item_grid(wt.total);
  if (g == 0) return hipSuccess;
#define LPC_POIS(BB, MM, CC) k_fft_x_poisson<BB, MM, CC><<<g, kFftNT, lds, s>>>(jobs, wt.offs, wt.njob, wt.total)
  if (chained) {
    if (B == 8 && M == 8) LPC_POIS(8, 8, true);
    else if (B == 8 && M == 12) LPC_POIS(8, 12, true);
    else if (B == 8 && M == 16) LPC_POIS(8, 16, true);
    else return hipErrorInvalidValue;
  }
  else if (B == 4 && M == 8) LPC_POIS(4, 8, false);
  else if (B == 8 && M == 8) LPC_POIS(8, 8, false);
  else if (B == 8 && M == 12) LPC_POIS(8, 12, false);
  else if (B == 8 && M == 16) LPC_POIS(8, 16, false);
  else if (B == 16 && M == 8) LPC_POIS(16, 8, false);
  else if (B == 16 && M == 12) LPC_POIS(16, 12, false);
  else if (B == 16 && M == 16) LPC_POIS(16, 16, false);
  else return hipErrorInvalidValue;
#undef LPC_POIS
  return hipGetLastError();
}

hipError_t launch_z_c2r(const ZC2RJob* jobs, WorkTable wt, int nc, int R, int P, size_t lds, hipStream_t s) {
  ensure_init();
  const unsigned g = item_grid(wt.total);
  if (g == 0) return hipSuccess;
#define LPC_ZC2R(NC, RR, PP) k_fft_z_c2r<NC, RR, PP><<<g, kFftNT, lds, s>>>(jobs, wt.offs, wt.njob, wt.total)
  if (nc == 1) {
    if (R == 8) LPC_ZC2R(1, 8, kEPT); else if (R == 16) LPC_ZC2R(1, 16, kEPT); else if (R == 32) LPC_ZC2R(1, 32, kEPT);
    else return hipErrorInvalidValue;
  } else if (nc == 3) {
    if (R == 4 && P == 8) LPC_ZC2R(3, 4, 8);
    else if (R == 4 && P == 12) LPC_ZC2R(3, 4, 12);
    else if (R == 4 && P == 16) LPC_ZC2R(3, 4, 16);
    else if (R == 8 && P == 8) LPC_ZC2R(3, 8, 8);
    else if (R == 8 && P == 12) LPC_ZC2R(3, 8, 12);
    else if (R == 8 && P == 16) LPC_ZC2R(3, 8, 16);
    else if (R == 16 && P == 8) LPC_ZC2R(3, 16, 8);
    else if (R == 16 && P == 12) LPC_ZC2R(3, 16, 12);
    else if (R == 16 && P == 16) LPC_ZC2R(3, 16, 16);
    else return hipErrorInvalidValue;
  } else {
    return hipErrorInvalidValue;
  }
#undef LPC_ZC2R
  return hipGetLastError();
}

}  // namespace kern
}  // namespace lpc
