// Device-side building blocks of liblpc's FFTs: complex helpers, radix-2/3/4/5/8/12 butterflies, one Stockham
// autosort stage over an LDS tile, and the XCD-aware workgroup remap. Included by the .hip sources only.
//
// An LDS tile holds B independent columns of one transform length n: element (j, b) at tile[j * BP + b] with
// BP >= B (n * B <= kTileElems). Stage s with radix R and current sub-transform length p (product of the
// earlier radices) reads x[i + r T] (T = n / R), multiplies by w^(r k) with w = exp(-+ 2 pi i / (p R)),
// k = i mod p, takes the length-R DFT and writes it to ((i - k) R + k + r p): the Stockham autosort ordering,
// so after the last stage the tile is in natural order. Each thread stages its butterflies in registers between two
// barriers, which makes the update in place.
#pragma once

#include <hip/hip_runtime.h>

#include "lpc_kernels.h"

namespace lpc {
namespace kern {

constexpr int kEPT = kTileElems / kFftNT;  // complex values per thread per stage (16)

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
__device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
__device__ __forceinline__ float2 cmulc(float2 a, float2 b) {
  return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
// multiply by -i (forward) or +i (inverse)
template <bool INV>
__device__ __forceinline__ float2 rot(float2 a) {
  return INV ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}

template <int R, bool INV>
struct Dft;

template <bool INV>
struct Dft<2, INV> {
  static __device__ __forceinline__ void run(float2* v) {
    float2 a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  }
};

template <bool INV>
struct Dft<4, INV> {
  static __device__ __forceinline__ void run(float2* v) {
    float2 t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
    float2 t2 = cadd(v[1], v[3]), t3 = rot<INV>(csub(v[1], v[3]));
    v[0] = cadd(t0, t2);
    v[2] = csub(t0, t2);
    v[1] = cadd(t1, t3);
    v[3] = csub(t1, t3);
  }
};

template <bool INV>
struct Dft<8, INV> {
  static __device__ __forceinline__ void run(float2* v) {
    float2 e[4] = {v[0], v[2], v[4], v[6]};
    float2 o[4] = {v[1], v[3], v[5], v[7]};
    Dft<4, INV>::run(e);
    Dft<4, INV>::run(o);
    const float h = 0.70710678118654752f;
    float2 o1 = cscale(cadd(o[1], rot<INV>(o[1])), h);   // w8^1 o1
    float2 o2 = rot<INV>(o[2]);                           // w8^2 o2
    float2 o3 = cscale(csub(rot<INV>(o[3]), o[3]), h);   // w8^3 o3
    v[0] = cadd(e[0], o[0]);
    v[4] = csub(e[0], o[0]);
    v[1] = cadd(e[1], o1);
    v[5] = csub(e[1], o1);
    v[2] = cadd(e[2], o2);
    v[6] = csub(e[2], o2);
    v[3] = cadd(e[3], o3);
    v[7] = csub(e[3], o3);
  }
};

template <bool INV>
struct Dft<3, INV> {
  static __device__ __forceinline__ void run(float2* v) {
    const float s3 = 0.86602540378443865f;
    float2 t = cadd(v[1], v[2]);
    float2 u = cscale(rot<INV>(csub(v[1], v[2])), s3);
    float2 m = csub(v[0], cscale(t, 0.5f));
    v[0] = cadd(v[0], t);
    v[1] = cadd(m, u);
    v[2] = csub(m, u);
  }
};

template <bool INV>
struct Dft<5, INV> {
  static __device__ __forceinline__ void run(float2* v) {
    const float c1 = 0.30901699437494742f, c2 = -0.80901699437494742f;
    const float s1 = 0.95105651629515357f, s2 = 0.58778525229247313f;
    float2 a1 = cadd(v[1], v[4]), b1 = csub(v[1], v[4]);
    float2 a2 = cadd(v[2], v[3]), b2 = csub(v[2], v[3]);
    float2 m1 = make_float2(v[0].x + c1 * a1.x + c2 * a2.x, v[0].y + c1 * a1.y + c2 * a2.y);
    float2 m2 = make_float2(v[0].x + c2 * a1.x + c1 * a2.x, v[0].y + c2 * a1.y + c1 * a2.y);
    float2 n1 = rot<INV>(make_float2(s1 * b1.x + s2 * b2.x, s1 * b1.y + s2 * b2.y));
    float2 n2 = rot<INV>(make_float2(s2 * b1.x - s1 * b2.x, s2 * b1.y - s1 * b2.y));
    v[0] = cadd(v[0], cadd(a1, a2));
    v[1] = cadd(m1, n1);
    v[4] = csub(m1, n1);
    v[2] = cadd(m2, n2);
    v[3] = csub(m2, n2);
  }
};

// 12 points as 4 x 3 by the prime-factor (Good-Thomas) mapping, which needs no twiddles because 4 and 3 are coprime:
// input n = (3 a + 4 b) mod 12 and output k = (9 a + 4 b) mod 12 for a < 4, b < 3, since n k = 3 a a' + 4 b b' mod 12.
// Four-point transforms over a for each b, then three-point transforms over b for each a.
template <bool INV>
struct Dft<12, INV> {
  static __device__ __forceinline__ void run(float2* v) {
    float2 y[3][4];
#pragma unroll
    for (int b = 0; b < 3; ++b) {
#pragma unroll
      for (int a = 0; a < 4; ++a) y[b][a] = v[(3 * a + 4 * b) % 12];
      Dft<4, INV>::run(y[b]);
    }
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      float2 z[3] = {y[0][a], y[1][a], y[2][a]};
      Dft<3, INV>::run(z);
#pragma unroll
      for (int b = 0; b < 3; ++b) v[(9 * a + 4 * b) % 12] = z[b];
    }
  }
};

// Thread geometry of a tile with B columns and row pitch BP: threads t < S B (S = kFftNT / B) own column
// b = t mod B and butterflies i = i0 + m S with i0 = t / B; the others idle during the stages.
struct TileGeom {
  int B, BP, S, b, i0;
  __device__ TileGeom(int B_, int BP_, int tid) : B(B_), BP(BP_), S(kFftNT / B_) {
    b = tid % B_;
    i0 = (tid < S * B_) ? tid / B_ : (1 << 30);
  }
};

// One Stockham stage over the tile (see the file comment). tws points at this stage's twiddles (k (R - 1) + r - 1).
// Requires n <= EPT S: each thread owns at most EPT points of its column, so ceil(EPT / R) butterflies (a kernel
// that knows a smaller bound than kEPT passes it, which sizes the register arrays down).
template <int R, bool INV, int EPT>
__device__ __forceinline__ void fft_stage(float2* tile, const float2* tws, int n, int p, int pmask, const TileGeom& g) {
  constexpr int MB = (EPT + R - 1) / R;
  const int T = n / R;
  float2 v[MB][R];
#pragma unroll
  for (int m = 0; m < MB; ++m) {
    const int i = g.i0 + m * g.S;
    if (i < T) {
      const float2* src = tile + i * g.BP + g.b;
#pragma unroll
      for (int r = 0; r < R; ++r) v[m][r] = src[r * T * g.BP];
    }
  }
  __syncthreads();
#pragma unroll
  for (int m = 0; m < MB; ++m) {
    const int i = g.i0 + m * g.S;
    if (i < T) {
      const int k = (pmask >= 0) ? (i & pmask) : (i % p);
      if (p > 1) {
        const float2* w = tws + k * (R - 1) - 1;
#pragma unroll
        for (int r = 1; r < R; ++r) {
          const float2 t = w[r];
          v[m][r] = INV ? cmulc(v[m][r], t) : cmul(v[m][r], t);
        }
      }
      Dft<R, INV>::run(v[m]);
      float2* dst = tile + ((i - k) * R + k) * g.BP + g.b;
#pragma unroll
      for (int r = 0; r < R; ++r) dst[r * p * g.BP] = v[m][r];
    }
  }
  __syncthreads();
}

// The same stage with the transform length N, the sub-transform length P and the tile geometry (B columns, pitch BP)
// known at compile time: the LDS offsets r T BP and r P BP become immediates and the twiddle index a constant mask.
template <int R, bool INV, int EPT, int N, int P, int B, int BP>
__device__ __forceinline__ void fft_stage_c(float2* tile, const float2* tws, int tid) {
  constexpr int MB = (EPT + R - 1) / R, T = N / R, S = kFftNT / B;
  const int b = tid % B;
  const int i0 = (tid < S * B) ? tid / B : (1 << 30);
  float2 v[MB][R];
#pragma unroll
  for (int m = 0; m < MB; ++m) {
    const int i = i0 + m * S;
    if (i < T) {
      const float2* src = tile + i * BP + b;
#pragma unroll
      for (int r = 0; r < R; ++r) v[m][r] = src[r * T * BP];
    }
  }
  __syncthreads();
#pragma unroll
  for (int m = 0; m < MB; ++m) {
    const int i = i0 + m * S;
    if (i < T) {
      const int k = ((P & (P - 1)) == 0) ? (i & (P - 1)) : (i % P);
      if (P > 1) {
        const float2* w = tws + k * (R - 1) - 1;
#pragma unroll
        for (int r = 1; r < R; ++r) {
          const float2 t = w[r];
          v[m][r] = INV ? cmulc(v[m][r], t) : cmul(v[m][r], t);
        }
      }
      Dft<R, INV>::run(v[m]);
      float2* dst = tile + ((i - k) * R + k) * BP + b;
#pragma unroll
      for (int r = 0; r < R; ++r) dst[r * P * BP] = v[m][r];
    }
  }
  __syncthreads();
}

// The first stage of a compile-time plan fed straight from global memory (sub-transform length 1: no twiddles), in
// two steps. first_stage_load issues the loads: butterfly i of column b takes rows i + r T (r < R) through load(row, b)
// into v. first_stage_store transforms them and writes the outputs to the tile at rows i R + r. No barrier: the caller
// synchronises before the next stage reads the tile.
template <int R, int EPT, int N, int B>
struct FirstStage {
  static constexpr int MB = (EPT + R - 1) / R, T = N / R, S = kFftNT / B;
  using Regs = float2[MB][R];
};
template <int R, int EPT, int N, int B, class Load>
__device__ __forceinline__ void first_stage_load(typename FirstStage<R, EPT, N, B>::Regs& v, Load load, int tid) {
  using F = FirstStage<R, EPT, N, B>;
  const int b = tid % B;
  const int i0 = (tid < F::S * B) ? tid / B : (1 << 30);
#pragma unroll
  for (int m = 0; m < F::MB; ++m) {
    const int i = i0 + m * F::S;
    if (i < F::T) {
#pragma unroll
      for (int r = 0; r < R; ++r) v[m][r] = load(i + r * F::T, b);
    }
  }
}
template <int R, bool INV, int EPT, int N, int B, int BP>
__device__ __forceinline__ void first_stage_store(float2* tile, typename FirstStage<R, EPT, N, B>::Regs& v, int tid) {
  using F = FirstStage<R, EPT, N, B>;
  const int b = tid % B;
  const int i0 = (tid < F::S * B) ? tid / B : (1 << 30);
#pragma unroll
  for (int m = 0; m < F::MB; ++m) {
    const int i = i0 + m * F::S;
    if (i < F::T) {
      Dft<R, INV>::run(v[m]);
      float2* dst = tile + i * R * BP + b;
#pragma unroll
      for (int r = 0; r < R; ++r) dst[r * BP] = v[m][r];
    }
  }
}

// Both steps, with mid() between them: all of a thread's loads are issued before mid() runs and before the first
// butterfly, so a caller can use mid() for work that overlaps them.
template <int R, bool INV, int EPT, int N, int B, int BP, class Load, class Mid>
__device__ __forceinline__ void fft_stage_from_global(float2* tile, Load load, Mid mid, int tid) {
  typename FirstStage<R, EPT, N, B>::Regs v;
  first_stage_load<R, EPT, N, B>(v, load, tid);
  mid();
  first_stage_store<R, INV, EPT, N, B, BP>(tile, v, tid);
}

// The same first stage for a tile whose columns come in pairs (b, b + B / 2) built from one source column: thread
// (i, bh) loads rows i + r T of source column bh once through load(row, bh), and pair(row, x) gives the value of
// column bh (column bh + B / 2 takes x itself). The loads of 16 rows x B / 2 columns per wave are each read once.
template <int R, int N, int B>
struct FirstStagePairs {
  static constexpr int BH = B / 2, T = N / R, S = kFftNT / BH, MB = (T + S - 1) / S;
  using Regs = float2[MB][R];
};
template <int R, int N, int B, class Load>
__device__ __forceinline__ void first_stage_pairs_load(typename FirstStagePairs<R, N, B>::Regs& x, Load load,
                                                       int tid) {
  using F = FirstStagePairs<R, N, B>;
  const int bh = tid % F::BH, i0 = tid / F::BH;
#pragma unroll
  for (int m = 0; m < F::MB; ++m) {
    const int i = i0 + m * F::S;
    if (i < F::T) {
#pragma unroll
      for (int r = 0; r < R; ++r) x[m][r] = load(i + r * F::T, bh);
    }
  }
}
template <int R, bool INV, int N, int B, int BP, class Pair>
__device__ __forceinline__ void first_stage_pairs_store(float2* tile, typename FirstStagePairs<R, N, B>::Regs& x,
                                                        Pair pair, int tid) {
  using F = FirstStagePairs<R, N, B>;
  const int bh = tid % F::BH, i0 = tid / F::BH;
#pragma unroll
  for (int m = 0; m < F::MB; ++m) {
    const int i = i0 + m * F::S;
    if (i < F::T) {
      float2 a[R];
#pragma unroll
      for (int r = 0; r < R; ++r) a[r] = pair(i + r * F::T, x[m][r]);
      Dft<R, INV>::run(a);
      Dft<R, INV>::run(x[m]);
      float2* dst = tile + i * R * BP + bh;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        dst[r * BP] = a[r];
        dst[r * BP + F::BH] = x[m][r];
      }
    }
  }
}
template <int R, bool INV, int N, int B, int BP, class Load, class Pair, class Mid>
__device__ __forceinline__ void fft_stage_from_global_pairs(float2* tile, Load load, Pair pair, Mid mid, int tid) {
  typename FirstStagePairs<R, N, B>::Regs x;
  first_stage_pairs_load<R, N, B>(x, load, tid);
  mid();
  first_stage_pairs_store<R, INV, N, B, BP>(tile, x, pair, tid);
}

// The last stage of a compile-time plan into registers: as fft_stage_c, but butterfly i of column b keeps its R
// outputs (rows (i - k) R + k + r P) in v instead of writing the tile. Each thread owns MB butterflies of one column,
// b = tid % B and i = tid / B + m kFftNT / B (m < MB), and they cover the stage exactly. No barrier after the tile
// reads.
template <int R, bool INV, int N, int P, int B, int BP, int MB>
__device__ __forceinline__ void fft_stage_to_regs(const float2* tile, const float2* tws, int tid,
                                                  float2 (&v)[MB][R]) {
  constexpr int T = N / R, S = kFftNT / B;
  static_assert(T == MB * S, "MB butterflies per thread cover the stage");
  const int b = tid % B, i0 = tid / B;
#pragma unroll
  for (int m = 0; m < MB; ++m) {
    const float2* src = tile + (i0 + m * S) * BP + b;
#pragma unroll
    for (int r = 0; r < R; ++r) v[m][r] = src[r * T * BP];
  }
#pragma unroll
  for (int m = 0; m < MB; ++m) {
    const int i = i0 + m * S;
    const int k = ((P & (P - 1)) == 0) ? (i & (P - 1)) : (i % P);
    if (P > 1) {
      const float2* w = tws + k * (R - 1) - 1;
#pragma unroll
      for (int r = 1; r < R; ++r) v[m][r] = INV ? cmulc(v[m][r], w[r]) : cmul(v[m][r], w[r]);
    }
    Dft<R, INV>::run(v[m]);
  }
}

// The first stage of a compile-time plan from registers (sub-transform length 1): butterfly i of column b takes its
// R inputs (rows i + r T) from v, and writes its DFT to the tile at rows i R + r. The same thread mapping as
// fft_stage_to_regs, so a stage that ends in registers can feed a transform whose first radix matches its last.
template <int R, bool INV, int N, int B, int BP, int MB>
__device__ __forceinline__ void fft_stage_from_regs(float2* tile, float2 (&v)[MB][R], int tid) {
  constexpr int T = N / R, S = kFftNT / B;
  static_assert(T == MB * S, "MB butterflies per thread cover the stage");
  const int b = tid % B, i0 = tid / B;
#pragma unroll
  for (int m = 0; m < MB; ++m) {
    Dft<R, INV>::run(v[m]);
    float2* dst = tile + (i0 + m * S) * R * BP + b;
#pragma unroll
    for (int r = 0; r < R; ++r) dst[r * BP] = v[m][r];
  }
}

// The last stage of a compile-time plan written straight to global memory: fft_stage_c with output row
// (i - k) R + k + r P going to store(row, b, value) instead of the tile. There is no barrier after the tile reads:
// nothing writes the tile again before the caller's next barrier.
template <int R, bool INV, int EPT, int N, int P, int B, int BP, class Store>
__device__ __forceinline__ void fft_stage_to_global(const float2* tile, const float2* tws, Store store, int tid) {
  constexpr int MB = (EPT + R - 1) / R, T = N / R, S = kFftNT / B;
  const int b = tid % B;
  const int i0 = (tid < S * B) ? tid / B : (1 << 30);
  float2 v[MB][R];
#pragma unroll
  for (int m = 0; m < MB; ++m) {
    const int i = i0 + m * S;
    if (i < T) {
      const float2* src = tile + i * BP + b;
#pragma unroll
      for (int r = 0; r < R; ++r) v[m][r] = src[r * T * BP];
    }
  }
#pragma unroll
  for (int m = 0; m < MB; ++m) {
    const int i = i0 + m * S;
    if (i < T) {
      const int k = ((P & (P - 1)) == 0) ? (i & (P - 1)) : (i % P);
      if (P > 1) {
        const float2* w = tws + k * (R - 1) - 1;
#pragma unroll
        for (int r = 1; r < R; ++r) {
          const float2 t = w[r];
          v[m][r] = INV ? cmulc(v[m][r], t) : cmul(v[m][r], t);
        }
      }
      Dft<R, INV>::run(v[m]);
      const int row = (i - k) * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) store(row + r * P, b, v[m][r]);
    }
  }
}

// A transform whose plan (radices Rs..., applied in order) and tile geometry are fixed at compile time. matches()
// tells whether a job's run-time plan is this one (then run() computes exactly what fft_tile computes, with the same
// twiddle table) and whether the tile geometry can hold it; kernels use it for the mesh sizes they are tuned for and
// fall back to fft_tile otherwise.
template <bool INV, int EPT, int B, int BP, int... Rs>
struct FixedFFT {
  static constexpr int kN = (Rs * ...);
  static constexpr int kNst = sizeof...(Rs);
  static constexpr bool kFits = kN <= EPT * (kFftNT / B) && kNst <= kMaxStages;
  template <class PL>
  static __device__ __forceinline__ bool matches(const PL& pl) {
    if constexpr (!kFits) {
      return false;
    } else {
      constexpr int radix[kNst] = {Rs...};
      if (pl.n != kN || pl.nst != kNst) return false;
#pragma unroll
      for (int s = 0; s < kNst; ++s)
        if (pl.radix[s] != radix[s]) return false;
      return true;
    }
  }
  template <int P, int R, int... More>
  static __device__ __forceinline__ void stages(float2* tile, const float2* tw, int tid) {
    fft_stage_c<R, INV, EPT, kN, P, B, BP>(tile, tw, tid);
    if constexpr (sizeof...(More) > 0) stages<P * R, More...>(tile, tw + P * (R - 1), tid);
  }
  // The caller has synchronised after filling the tile.
  static __device__ __forceinline__ void run(float2* tile, const float2* tw, int tid) {
    if constexpr (kFits) stages<1, Rs...>(tile, tw, tid);
  }
  // With GIN the first stage reads global memory through load (the tile is not filled first; mid runs while the
  // loads are in flight); with GOUT the last stage writes global memory through store (the tile keeps the last
  // stage's input). Without them the stage works in the tile as in run(). Plans of two stages or more.
  template <bool GIN, bool GOUT, bool PAIRS, int P, int R, int... More, class Load, class Pair, class Mid, class Store>
  static __device__ __forceinline__ void io_stages(float2* tile, const float2* tw, int tid, Load load, Pair pair,
                                                   Mid mid, Store store) {
    if constexpr (P == 1 && GIN) {
      if constexpr (PAIRS)
        fft_stage_from_global_pairs<R, INV, kN, B, BP>(tile, load, pair, mid, tid);
      else
        fft_stage_from_global<R, INV, EPT, kN, B, BP>(tile, load, mid, tid);
      __syncthreads();
    } else if constexpr (sizeof...(More) == 0 && GOUT) {
      fft_stage_to_global<R, INV, EPT, kN, P, B, BP>(tile, tw, store, tid);
    } else {
      fft_stage_c<R, INV, EPT, kN, P, B, BP>(tile, tw, tid);
    }
    if constexpr (sizeof...(More) > 0)
      io_stages<GIN, GOUT, PAIRS, P * R, More...>(tile, tw + P * (R - 1), tid, load, pair, mid, store);
  }
  // PAIRS: the tile's columns come in pairs built from one loaded column (fft_stage_from_global_pairs)
  template <bool GIN, bool GOUT, bool PAIRS, class Load, class Pair, class Mid, class Store>
  static __device__ __forceinline__ void run_io(float2* tile, const float2* tw, int tid, Load load, Pair pair, Mid mid,
                                                Store store) {
    if constexpr (kFits && kNst >= 2) io_stages<GIN, GOUT, PAIRS, 1, Rs...>(tile, tw, tid, load, pair, mid, store);
  }
};

// All stages of plan `pl` over the B columns of the tile (row pitch BP). tw is the plan's per-stage twiddle
// table. The caller has synchronised after filling the tile. With R12 false the radix-12 stage is not compiled in
// (for a kernel at its register cap): the plan must then come from make_plan(n, p, false).
template <bool INV, int EPT = kEPT, bool R12 = true, class PL>
__device__ __forceinline__ void fft_tile(float2* tile, const float2* tw, const PL& pl, int B, int BP, int tid) {
  const TileGeom g(B, BP, tid);
  const int n = pl.n;
  for (int s = 0; s < pl.nst; ++s) {
    const float2* tws = tw + pl.tw_off[s];
    const int p = pl.p[s], pm = pl.pmask[s];
    switch (pl.radix[s]) {  // the plans use radices 8, 4, 2, 12, 3 and 5 (make_plan)
      case 8: fft_stage<8, INV, EPT>(tile, tws, n, p, pm, g); break;
      case 12:
        if constexpr (R12) fft_stage<12, INV, EPT>(tile, tws, n, p, pm, g);
        break;
      case 4: fft_stage<4, INV, EPT>(tile, tws, n, p, pm, g); break;
      case 2: fft_stage<2, INV, EPT>(tile, tws, n, p, pm, g); break;
      case 3: fft_stage<3, INV, EPT>(tile, tws, n, p, pm, g); break;
      default: fft_stage<5, INV, EPT>(tile, tws, n, p, pm, g); break;
    }
  }
}


// Row pitch of a strided tile of B columns, whose lanes run along the columns: 8-column tiles are left unpadded
// (with a pitch of 9, two rows met in one 16-lane group of a 64-bit LDS access share banks; a model of the stage
// accesses gives 1.9x the conflict-free cycles for pitch 9 and 1.1x for pitch 8), wider tiles take B + 1.
__host__ __device__ constexpr int strided_pitch(int B) { return B == 8 ? 8 : B + 1; }

// Copy `count` <= 2 kFftNT entries (tables of lengths up to 1024, the largest mesh side) of a precomputed table from
// global memory to LDS in two steps: table_load issues the loads into registers, table_store writes them (no
// barrier). A kernel issues its tables' loads before its data loads, so that writing the tables waits for them only
// (a load-then-store loop would wait out one memory latency per table, behind every load issued before it).
template <class T>
struct TableRegs {
  T v[2];
};
template <class T>
__device__ __forceinline__ TableRegs<T> table_load(const T* __restrict__ src, int count, int tid) {
  LPC_GLOBAL const T* g = to_global(src);
  TableRegs<T> r;
#pragma unroll
  for (int m = 0; m < 2; ++m) {
    const int i = tid + m * kFftNT;
    if (i < count) r.v[m] = g[i];
  }
  return r;
}
template <class T>
__device__ __forceinline__ void table_store(T* dst, const TableRegs<T>& r, int count, int tid) {
#pragma unroll
  for (int m = 0; m < 2; ++m) {
    const int i = tid + m * kFftNT;
    if (i < count) dst[i] = r.v[m];
  }
}


}  // namespace kern
}  // namespace lpc
