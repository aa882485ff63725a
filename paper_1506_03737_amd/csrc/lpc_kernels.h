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

// One 1-D transform length factored into radix stages (applied in order; radices 2, 3, 4, 5, 8, 12). For stage s,
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

// Stages of a length-n transform: radix 8 (2, 4 for the rest of the power of two), 3 and 5; with radix12 a radix-4
// and a radix-3 stage become one radix-12 stage. False if n has a prime factor > 5 or n < 1.
bool make_plan(int n, Plan1D* p, bool radix12 = true);
// The plan of the same length with the radices applied in reverse order (p, pmask and tw_off recomputed).
Plan1D reversed_plan(const Plan1D& p);
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

// On-the-fly lightcone of one drift a_i -> a_{i+1} (Sec. 6.1, 6.2). Particle images that leave the lightcone in the
// drift are appended to `out` (the count in *count, records past `capacity` dropped).
constexpr int kLcTab = 65;       // nodes of the partial-drift table over t = (a - a_i) / (a_{i+1} - a_i) in [0, 1]
constexpr int kLcList = 512;     // replicate images a workgroup keeps after its own culling (more: test them all)
struct LcRecord {                // layout of lpc_lightcone_record
  float pos[3];
  float vel[3];
  float a;
  int index;
  int replicate;
  int reserved;
};
struct LightconeStep {
  float ai, aip1;                // a_i, a_{i+1}
  float rli, rln;                // R_L(a_i), R_L(a_{i+1}) (Mpc/h)
  float ox, oy, oz;              // observer (Mpc/h)
  float f1h, f2h;                // frame momentum factors at a_{i+1/2} (0 for plain PM)
  const float* tab;              // [kLcTab][3]: Q(a_i, a), D1(a) - D1(a_i), D2(a) - D2(a_i) at the nodes
  const int* reps;               // [nrep][4]: replicate (i, j, k) and its flat index
  int nrep;
  LcRecord* out;
  unsigned long long* count;
  long long capacity;
};

hipError_t fill_i32(int* p, size_t count, int value, hipStream_t s);

// ---------------------------------------------------------------------------------------------------------------
// Batched stage launches. Every stage kernel runs over the items of a work table: FFT kernels take one item per
// workgroup (w = blockIdx.x); the particle kernels are launched with one workgroup per item too, and their loops
// walk w = blockIdx.x, blockIdx.x + G, ... (so any grid of G workgroups is correct). Item w belongs to job j with
// offs[j] <= w < offs[j + 1]
// (offs has njob + 1 entries, offs[0] = 0, offs[njob] = total, every offs[j] a multiple of 8 so that items keep their
// XCD position within a job). A single box is a batch of one job. Job arrays and offsets live in device memory.
// Pointers read from job tables are generic; casting them to the global address space lets the compiler issue
// global (not flat) memory instructions for them, as it does for pointer kernel arguments.
// (The host pass of hipcc also parses kernel bodies; there the qualifiers are dropped.)
#if defined(__HIP_DEVICE_COMPILE__)
#define LPC_GLOBAL __attribute__((address_space(1)))
#define LPC_CONST __attribute__((address_space(4)))
#else
#define LPC_GLOBAL
#define LPC_CONST
#endif
template <class T>
__device__ __forceinline__ LPC_GLOBAL T* to_global(T* p) {
  return (LPC_GLOBAL T*)p;
}
// Job tables are written before a launch and only read by it: reading them through the constant address space
// lets the compiler use scalar loads and reload fields instead of holding them in registers across a work loop.
template <class T>
__device__ __forceinline__ const LPC_CONST T* to_const(const T* p) {
  return (const LPC_CONST T*)p;
}

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own L2). Remap the hardware block index so
// that each XCD receives a contiguous range of logical tiles: neighbouring tiles (which share cache lines at their
// edges) then run on the same XCD.
// Periodic wrap of a coordinate that moved by less than one box into [0, box). x + box can round up to box itself
// in FP32 when x is a tiny negative number; that point is the periodic image of 0, which is returned instead.
__device__ __forceinline__ float wrap_box(float x, float box) {
  if (x >= box) x -= box;
  if (x < 0.f) {
    x += box;
    if (x >= box) x = 0.f;
  }
  return x;
}

__device__ __forceinline__ int xcd_remap(int bid, int nblocks) {
  const int per = nblocks / 8, rem = nblocks % 8;
  const int xcd = bid % 8, local = bid / 8;
  return xcd * per + min(xcd, rem) + local;
}

// XCD-contiguous chunks of C items: XCD x (which takes the blocks b = x mod 8) processes the chunks 8 c + x, c = 0,
// 1, ..., so at any time the eight XCDs work on eight adjacent chunks rather than on eight distant eighths of the
// items. Items past the last whole group of 8 C take xcd_remap's order. A permutation of [0, n) for n a multiple of 8.
__device__ __forceinline__ int xcd_chunk_remap(int bid, int n, int C) {
  const int full = n / (8 * C) * (8 * C);
  if (bid >= full) return full + xcd_remap(bid - full, n - full);
  const int x = bid % 8, k = bid / 8;
  return ((k / C) * 8 + x) * C + k % C;
}

struct WorkTable {
  const int* offs;
  int njob;
  int total;
};

// Mesh tiles of the particle sort and of the tiled deposit: kTX x kTY x kTZ cells (x, y, z; narrower at the end of
// an axis they do not divide). 32 cells along z make every row of a tile one 128-byte line of the FP32 density, and
// kTY kTZ = kNT puts one thread on each (y, z) cell of a tile plane. A box has ntx ny nz = ceil(Nm / kTX),
// ceil(Nm / kTY), ceil(Nm / kTZ) tiles; tile (tx, ty, tz) has index t = (tx nty + ty) ntz + tz and two buckets, 2 t
// (interior) and 2 t + 1 (boundary: the particle's cell is in the tile's last layer along some axis); one extra bucket
// (2 ntx nty ntz) collects particles whose position is unusable.
constexpr int kTX = 16, kTY = 8, kTZ = 32;
struct TileGrid {
  int x, y, z;
  int count() const { return x * y * z; }
};
inline TileGrid tile_grid(int nm) { return TileGrid{(nm + kTX - 1) / kTX, (nm + kTY - 1) / kTY, (nm + kTZ - 1) / kTZ}; }

struct SortJob {        // key pass and scatter of one box: src (SoA [3][n]) -> dst in tile order
  const float* pos;
  const float* vel;     // vel / psi1 / psi2 are carried only when the dst pointer is not NULL
  const float* psi1;
  const float* psi2;
  const int* orig;      // index in the caller's arrays; NULL when src is the caller's arrays (orig = i)
  float* dpos;
  float* dvel;
  float* dpsi1;
  float* dpsi2;
  int* dorig;
  int64_t n, pbase;     // particles; first global particle index of the box (key / rank arrays)
  int tbase, nm;        // first global tile index; mesh size
  int ntx, nty, ntz;    // tiles along x, y, z
  double scale;         // nm 2^16 / box
};
// ceil(2^32 / d) for d > 1, 0 for d = 1: the reciprocal with which t / d = mulhi(t, inv) for t < 2^32 / d
inline uint32_t div_inverse(int d) {
  return d <= 1 ? 0u : static_cast<uint32_t>(((uint64_t(1) << 32) + static_cast<uint64_t>(d) - 1) / static_cast<uint64_t>(d));
}

struct DepJob {         // tiled deposit of one box from its tile-sorted positions
  const float* pos;
  int64_t n, pbase;
  int tbase, nm;
  int ntx, nty, ntz;
  uint32_t inv_yz, inv_z;  // div_inverse(nty ntz), div_inverse(ntz): tiles number fewer than 2^32 / (nty ntz)
  double scale;
  uint64_t* dens;       // int64 counts, or NULL
  float* delta;         // FP32 density contrast C mscale - 1, or NULL
  double mscale;
};
struct UnsortJob {      // sorted pos / vel back to the caller's order
  const float* spos;
  const float* svel;
  const int* orig;
  float* pos;
  float* vel;
  int64_t n;
};
struct PartJob {        // one box's particles and meshes
  float* pos;
  float* vel;
  const float* psi1;
  const float* psi2;
  int64_t n;
  uint64_t* dens;       // fixed-point counts (deposit)
  const float* force;   // AoS float3 force mesh (gather)
  float* grad;          // gather output [3][n] (pm force only), written at index orig[i]
  const int* orig;      // caller's index of each (sorted) particle; NULL = identity
  int nm;
  float box;
  double scale;         // nm 2^16 / box
  int64_t pbase;        // first global particle index of the box (key / rank arrays of the next sort)
  int tbase;            // first global tile index of the box
  int ntx, nty, ntz;    // tiles along x, y, z
};
// FFT tables (device, built once per call on the host in FP64 and rounded to FP32): tw = the plan's stage twiddles
// (Plan1D), roots[k] = exp(-2 pi i k / n) for k <= n / 2 (real-transform split), win[m] = sinc^2(pi m / n) for
// m <= n / 2 (CIC window).
struct ZR2CJob {        // forward z pass of one mesh
  const void* in;       // uint64 counts (fixed) or FP32 reals
  float2* out;
  const float2 *tw, *roots;
  double mscale;        // fixed point: delta = C mscale - 1
  int n, nrows, pitch;
  Plan1D pl;            // length n / 2
};
struct AxisJob {        // complex FFT along a strided axis, ncomp meshes
  float2* base;
  const float2* tw;
  int64_t astr, ostr, cstr;
  int n, ncols, ntc, per_comp;  // per_comp = n_outer * ntc tiles (rounded up to 8)
  Plan1D pl;
};
struct PoissonJob {     // fused forward x / Poisson-gradient / inverse x of one box
  float2 *A, *B, *C;
  const float2* tw;
  const float2* tw_rev;  // stage twiddles of the plan with its radices in reverse order (reversed_plan)
  const float* win;
  int nm, pitch, ntc, deconv;
  float kf, inv_m3;
  Plan1D pl;
};
struct YGradJob {       // inverse y pass of the force: A in place; i k_y psi (from C) into B, psi back into C
  float2 *A, *B, *C;
  const float2* tw;
  int64_t astr, ostr;   // stride along y, stride of the outer (x) index
  int n, ncols;
  int ntc, per_comp;    // component 0: column tiles of B per row, items (a multiple of 8)
  int ntc1, per_comp1;  // component 1: column tiles of B / 2 per row, items (a multiple of 8)
  float kf;             // 2 pi / L
  Plan1D pl;
};
struct ZC2RJob {        // inverse z pass of NC spectra of one mesh
  const float2 *in0, *in1, *in2;
  float* out;
  const float2 *tw, *roots;
  float kz3;            // if nonzero (NC = 3): the third spectrum is psi, taken as i k_z psi with k_z = kz3 k
  int n, nrows, pitch;
  float scale;
  Plan1D pl;            // length n / 2
};

// Tile geometry chosen for one transform length (shared by the host builder and the launchers).
int strided_cols(int n);          // B of strided passes
int z_rows(int n, int nc);        // rows per z-pass tile for nc interleaved spectra
// Tile widths the FFT kernels are instantiated for, and whether width w fits length n (stage and load capacity of a
// tile, 160 KiB of LDS).
enum class TileKind { kZRows, kAxisCols, kPoissonCols, kForceC2RRows };
bool tile_ok(TileKind kind, int n, int w);
size_t lds_z_r2c(int n, int B);
size_t lds_axis(int n, int B);
int axis_points(int n, int B);     // points per thread of a strided tile of B columns (8, 12 or 16)
int r2c_points(int n, int B);      // points per thread of a forward r2c z tile of B rows (8, 12 or 16)
int c2r_points(int n, int R);      // points per thread of a three-spectrum c2r z tile of R rows (8, 12 or 16)
int poisson_points(int n, int B);  // points per thread of a fused x + Poisson tile (8, 12 or 16)
size_t lds_x_poisson(int n, int B, int M, bool chained);
size_t lds_z_c2r(int n, int B);

hipError_t launch_tile_key(const SortJob* jobs, WorkTable wt, int* cnt, int* key, int* rank, int* flags,
                           hipStream_t s);
int scan_blocks(int count);  // entries of the block-sum scratch of launch_scan
hipError_t launch_scan(const int* cnt, int* start, int count, int* block_sums, hipStream_t s);  // start: count + 1
hipError_t launch_scatter(const SortJob* jobs, WorkTable wt, const int* key, const int* rank, const int* start,
                          hipStream_t s);
hipError_t launch_deposit_tiles(const DepJob* jobs, WorkTable wt, const int* start, int* flags, hipStream_t s);
hipError_t launch_unsort(const UnsortJob* jobs, WorkTable wt, hipStream_t s);
// With key != NULL the kernel also does the next sort's key pass on the positions it writes (bucket, rank via cnt,
// which must be zero): the key pass of k_tile_key folded into the drift.
hipError_t launch_gather_kick_drift(const PartJob* jobs, WorkTable wt, KickDrift kd, int* flags, int* cnt, int* key,
                                    int* rank, hipStream_t s);
// The same kernel with the lightcone test of Sec. 6.1 in its drift (kd.do_drift must be 1).
hipError_t launch_gather_kick_drift_lc(const PartJob* jobs, WorkTable wt, KickDrift kd, const LightconeStep& lc,
                                       int* flags, int* cnt, int* key, int* rank, hipStream_t s);
hipError_t launch_gather(const PartJob* jobs, WorkTable wt, int* flags, hipStream_t s);
hipError_t launch_frame(const PartJob* jobs, WorkTable wt, float f1, float f2, hipStream_t s);
// B: tile columns (rows for z passes); lds: dynamic LDS bytes (the max over the jobs).
// One-time kernel attribute set-up (large dynamic LDS); launches do it themselves, graph capture calls it first.
void init_kernels();
hipError_t launch_z_r2c(const ZR2CJob* jobs, WorkTable wt, bool fixed, int B, int P, size_t lds, int* flags,
                        hipStream_t s);
hipError_t launch_axis(const AxisJob* jobs, WorkTable wt, bool inverse, int B, int P, size_t lds, hipStream_t s);
hipError_t launch_y_grad(const YGradJob* jobs, WorkTable wt, int B, int P, size_t lds, hipStream_t s);
// chained: every job's plan is poisson_chainable and B = 8 (the transforms chained through registers)
hipError_t launch_poisson(const PoissonJob* jobs, WorkTable wt, int B, int M, bool chained, size_t lds, hipStream_t s);
// Plans 8 x 8 x R with R in {12, 5, 4, 3}, and 4 x 4 x 8 x 8: the fused x pass can chain its transforms through
// registers.
bool poisson_chainable(const Plan1D& pl);
hipError_t launch_z_c2r(const ZC2RJob* jobs, WorkTable wt, int nc, int R, int P, size_t lds, hipStream_t s);

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
// Primordial non-Gaussianity (Sec. 5): phi_hat from the noise spectrum; D^s spectral multipliers; the real-space sum
// of the products of a group of terms; delta_L_hat = alpha0 k^2 T(k) (phi_hat + fNL NL_hat).
constexpr int kPngMaxTerms = 4;
struct PngProducts {  // out[i] = sum_t c[t] fa[t][i] fb[t][i]
  float* out;
  const float* fa[kPngMaxTerms];
  const float* fb[kPngMaxTerms];
  float c[kPngMaxTerms];
  int n;
};
hipError_t png_potential(float2* spec, int N, int pitch, double box, double a_phi, double n_s, hipStream_t s);
hipError_t png_power(const float2* in, float2* out, int N, int pitch, double box, double expo, double coef,
                     bool accumulate, hipStream_t s);
hipError_t png_products(const PngProducts& pp, int64_t count, hipStream_t s);
hipError_t png_to_delta(float2* phi, const float2* nl, int N, int pitch, double box, double f_nl, double alpha0,
                        double omega_m, double h, hipStream_t s);
hipError_t ic_assemble(float* pos, float* vel, int32_t* id, const float* psi1, const float* psi2, int N, double box,
                       float d1, float d2, float f1, float f2, hipStream_t s);

// Power-spectrum binning of a half spectrum: sums[b] += (k, P) per mode, counts[b] += multiplicity.
// Reduced-bispectrum pieces (FFT shell estimator). A shell is klo <= |k| < khi. shell_fill writes a whole half
// spectrum (pitch included): delta_hat / W in the shell (or 1 with indicator), 0 elsewhere. triple_sum and
// shell_power write sum_blocks() FP64 partial sums each: sum a b c over M cells; sum of mult |delta_hat|^2 / W^2 and
// of mult over the shell's modes (mult 2 off the kz = 0 and Nyquist planes).
hipError_t shell_fill(const float2* spec, float2* out, int nm, int pitch, double box, double klo, double khi,
                      bool indicator, hipStream_t s);
hipError_t triple_sum(const float* a, const float* b, const float* c, int64_t M, double* part, hipStream_t s);
hipError_t shell_power(const float2* spec, int nm, int pitch, double box, double klo, double khi, double* part_p,
                       double* part_n, hipStream_t s);
int sum_blocks();
hipError_t pk_bin(const float2* spec, int nm, int pitch, double box, double k_max, int n_bins, double pscale,
                  double* sums, unsigned long long* counts, hipStream_t s);

}  // namespace kern
}  // namespace lpc
