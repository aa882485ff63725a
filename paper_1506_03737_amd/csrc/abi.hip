// C ABI of liblpc (declared in include/lpc.h): argument checks, the workspace plan, the FP64 coefficient table and
// the sequence of kernel launches for each entry point. No C++ exception crosses this boundary.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstddef>
#include <cstdio>
#include <cstring>
#include <exception>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/lpc.h"
#include "abi_common.h"
#include "lpc_host.h"
#include "lpc_kernels.h"

namespace {
thread_local std::string g_error;
}  // namespace

static_assert(sizeof(lpc_lightcone_record) == sizeof(lpc::kern::LcRecord), "lightcone record layout");
static_assert(offsetof(lpc_lightcone_record, a) == offsetof(lpc::kern::LcRecord, a), "lightcone record layout");
static_assert(offsetof(lpc_lightcone_record, replicate) == offsetof(lpc::kern::LcRecord, replicate),
              "lightcone record layout");

namespace lpc {
namespace abi {

lpc_status fail(lpc_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_error = buf;
  return s;
}

const char* last_error() { return g_error.c_str(); }

}  // namespace abi
}  // namespace lpc

namespace {

using lpc::abi::HipError;
using lpc::abi::check;
using lpc::abi::fail;
using lpc::abi::guarded;
using lpc::kern::Plan1D;
namespace kern = lpc::kern;
namespace host = lpc::host;

// Optional per-stage timing: when enabled, every kernel launch of an entry point is bracketed by HIP events on the
// call's stream; the durations are read after the call's final synchronisation and accumulated per stage name.
struct StageStat {
  long long launches = 0;
  double total_ms = 0.0;
};
struct Profiler {
  bool on = false;
  std::vector<std::pair<std::string, StageStat>> stats;  // insertion-ordered
  std::vector<hipEvent_t> free_events;
  struct Pending {
    const char* name;
    hipEvent_t a, b;
  };
  std::vector<Pending> pending;
  hipEvent_t get() {
    if (!free_events.empty()) {
      hipEvent_t e = free_events.back();
      free_events.pop_back();
      return e;
    }
    hipEvent_t e;
    check(hipEventCreate(&e), "hipEventCreate");
    return e;
  }
  StageStat& stat(const char* name) {
    for (auto& kv : stats)
      if (kv.first == name) return kv.second;
    stats.emplace_back(name, StageStat{});
    return stats.back().second;
  }
  // called after the stream has been synchronised
  void collect() {
    for (auto& p : pending) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
        StageStat& st = stat(p.name);
        st.launches += 1;
        st.total_ms += ms;
      }
      free_events.push_back(p.a);
      free_events.push_back(p.b);
    }
    pending.clear();
  }
};
Profiler g_prof;

// Launch one stage through its launcher `f` (returning hipError_t), timed when profiling is on.
template <class F>
void stage(const char* name, hipStream_t s, F f) {
  if (!g_prof.on) {
    check(f(), name);
    return;
  }
  hipEvent_t a = g_prof.get(), b = g_prof.get();
  check(hipEventRecord(a, s), "hipEventRecord");
  check(f(), name);
  check(hipEventRecord(b, s), "hipEventRecord");
  g_prof.pending.push_back({name, a, b});
}

constexpr size_t kAlign = 256;
size_t round_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }
int round8(int x) { return (x + 7) / 8 * 8; }

bool fft_size_ok(int n) {
  if (n < 8 || n > 1024 || (n % 2) != 0) return false;
  Plan1D p;
  return kern::make_plan(n, &p) && kern::make_plan(n / 2, &p);
}

constexpr size_t kJobRegion = size_t(1) << 20;  // device bytes reserved for the job tables of one call

// Particle storage of a call (after the meshes): tile-sorted copies of every box's particles (two copies for a COLA
// run, ping-ponged by the per-step re-sort, with pos, vel, psi1, psi2 and the caller's index; one copy with pos and
// the caller's index for a single force or spectrum), sort keys and ranks, and the tile counts and starts.
struct BoxParts {
  float *pos = nullptr, *vel = nullptr, *psi1 = nullptr, *psi2 = nullptr;
  int* orig = nullptr;
};
struct SortSpace {
  std::vector<BoxParts> copy[2];
  std::vector<int64_t> pbase;
  std::vector<int> tbase;
  std::vector<kern::TileGrid> nt;
  int *key = nullptr, *rank = nullptr, *cnt = nullptr, *start = nullptr, *block_sums = nullptr;
  int G = 0;  // buckets over all boxes (2 tiles + 1 each)
};

// Lays out the sort space of boxes with particle counts n[] and meshes nm[] from workspace offset `off` (base NULL:
// sizes only) and returns the end offset.
size_t layout_sort(char* base, size_t off, const std::vector<int64_t>& n, const std::vector<int>& nm, bool cola,
                   SortSpace* out) {
  auto take = [&off](size_t bytes) {
    const size_t at = off;
    off += round_up(bytes);
    return at;
  };
  auto ptr = [base](size_t at) { return base ? base + at : nullptr; };
  SortSpace ss;
  int64_t ptot = 0;
  int G = 0;
  for (size_t b = 0; b < n.size(); ++b) {
    ss.pbase.push_back(ptot);
    ss.tbase.push_back(G);
    const kern::TileGrid nt = kern::tile_grid(nm[b]);
    ss.nt.push_back(nt);
    ptot += n[b];
    G += 2 * nt.count() + 1;
  }
  for (int c = 0; c < (cola ? 2 : 1); ++c) {
    for (size_t b = 0; b < n.size(); ++b) {
      const size_t v3 = sizeof(float) * 3 * static_cast<size_t>(n[b]);
      BoxParts bp;
      bp.pos = reinterpret_cast<float*>(ptr(take(v3)));
      if (cola) {
        bp.vel = reinterpret_cast<float*>(ptr(take(v3)));
        bp.psi1 = reinterpret_cast<float*>(ptr(take(v3)));
        bp.psi2 = reinterpret_cast<float*>(ptr(take(v3)));
      }
      bp.orig = reinterpret_cast<int*>(ptr(take(sizeof(int) * static_cast<size_t>(n[b]))));
      ss.copy[c].push_back(bp);
    }
  }
  ss.key = reinterpret_cast<int*>(ptr(take(sizeof(int) * static_cast<size_t>(ptot))));
  ss.rank = reinterpret_cast<int*>(ptr(take(sizeof(int) * static_cast<size_t>(ptot))));
  ss.cnt = reinterpret_cast<int*>(ptr(take(sizeof(int) * static_cast<size_t>(G))));
  ss.start = reinterpret_cast<int*>(ptr(take(sizeof(int) * (static_cast<size_t>(G) + 1))));
  ss.block_sums = reinterpret_cast<int*>(ptr(take(sizeof(int) * static_cast<size_t>(kern::scan_blocks(G)))));
  ss.G = G;
  if (out) *out = ss;
  return off;
}

// Workspace plan of one operation on an n^3 mesh with np particles: flags, the job-table region, the meshes, then
// the sort space, every region 256-byte aligned.
struct Plan {
  size_t flags = 0, jobs = 0, dens = 0, A = 0, B = 0, C = 0, bins = 0, sort = 0, total = 0;
  size_t fields = 0;  // three real meshes (bispectrum)
};

// Triangles per lpc_bispectrum call (their partial sums share one workspace region)
constexpr int kMaxTriangles = 256;
// FP64 partial sums per triangle: the filtered and indicator triple sums, the three shells' power and mode counts
constexpr int kPartsPerTriangle = 8;

Plan make_ws_plan(int n, int op, int64_t np) {
  Plan p;
  const size_t M = static_cast<size_t>(n) * n * n;
  const size_t cbytes = round_up(static_cast<size_t>(n) * n * kern::mesh_pitch(n) * sizeof(float2));
  size_t off = round_up(sizeof(int) * kern::kNumFlags);
  auto take = [&off](size_t bytes) {
    size_t at = off;
    off += round_up(bytes);
    return at;
  };
  p.jobs = take(kJobRegion);
  switch (op) {
    case LPC_OP_PM_FORCE:
    case LPC_OP_COLA_STEP:
      p.dens = take(M * 12);  // int64 counts, later the AoS float3 force mesh
      p.A = take(cbytes);
      p.B = take(cbytes);
      p.C = take(cbytes);
      break;
    case LPC_OP_INIT_IC:
      p.A = take(cbytes);
      p.B = take(cbytes);
      p.C = take(cbytes);  // the non-linear term's spectrum of a non-Gaussian field
      break;
    case LPC_OP_POWER_SPECTRUM:
      p.dens = take(M * 8);
      p.A = take(cbytes);
      p.bins = take(static_cast<size_t>(2048) * 3 * sizeof(double));
      break;
    case LPC_OP_BISPECTRUM:
      p.dens = take(M * 8);
      p.A = take(cbytes);  // delta_hat
      p.B = take(cbytes);  // a shell-filtered spectrum, consumed by its inverse transform
      p.fields = take(M * 3 * sizeof(float));
      p.bins = take(static_cast<size_t>(kMaxTriangles) * kPartsPerTriangle * kern::sum_blocks() * sizeof(double));
      break;
    case LPC_OP_FFT:
      break;
    default:
      return Plan{};
  }
  if (op == LPC_OP_PM_FORCE || op == LPC_OP_COLA_STEP || op == LPC_OP_POWER_SPECTRUM || op == LPC_OP_BISPECTRUM) {
    p.sort = off;
    off = layout_sort(nullptr, off, {np}, {n}, op == LPC_OP_COLA_STEP, nullptr);
  }
  p.total = off;
  return p;
}

SortSpace sort_space(void* ws, const Plan& p, int n, int op, int64_t np) {
  SortSpace ss;
  layout_sort(static_cast<char*>(ws), p.sort, {np}, {n}, op == LPC_OP_COLA_STEP, &ss);
  return ss;
}

lpc_status check_ws(void* ws, size_t ws_bytes, size_t need) {
  if (ws == nullptr) return fail(LPC_ERR_INVALID_ARG, "workspace pointer is NULL");
  if (reinterpret_cast<uintptr_t>(ws) % kAlign != 0) return fail(LPC_ERR_WORKSPACE, "workspace not 256-byte aligned");
  if (ws_bytes < need)
    return fail(LPC_ERR_WORKSPACE, "workspace too small: %zu bytes given, %zu needed", ws_bytes, need);
  return LPC_OK;
}

lpc_status check_mesh(int nm, const char* what) {
  if (!fft_size_ok(nm))
    return fail(LPC_ERR_UNSUPPORTED_SIZE, "%s = %d: need an even size in [8, 1024] whose prime factors are 2, 3, 5",
                what, nm);
  return LPC_OK;
}

// FFT tile widths per mesh size: the built-in rule, and overrides set through lpc_fft_tiling_set.
lpc_fft_tiling default_tiling(int n) {
  lpc_fft_tiling t;
  t.z_rows = std::max(8, kern::z_rows(n, 1));
  t.axis_cols = kern::strided_cols(n);
  t.poisson_cols = std::min(16, kern::strided_cols(n));
  t.c2r_rows = std::max(4, std::min(16, kern::z_rows(n, 3)));
  return t;
}

struct TilingTable {
  std::mutex mu;
  std::map<int, lpc_fft_tiling> over;
  uint64_t generation = 0;  // bumped on every change, part of the batched graph's key
};
TilingTable g_tiling;

lpc_fft_tiling tiling_of(int n) {
  std::lock_guard<std::mutex> lock(g_tiling.mu);
  const auto it = g_tiling.over.find(n);
  return it != g_tiling.over.end() ? it->second : default_tiling(n);
}

uint64_t tiling_generation() {
  std::lock_guard<std::mutex> lock(g_tiling.mu);
  return g_tiling.generation;
}

lpc_status check_tiling(int n, const lpc_fft_tiling& t) {
  const struct {
    kern::TileKind kind;
    int w;
    const char* name;
  } fields[] = {{kern::TileKind::kZRows, t.z_rows, "z_rows"},
                {kern::TileKind::kAxisCols, t.axis_cols, "axis_cols"},
                {kern::TileKind::kPoissonCols, t.poisson_cols, "poisson_cols"},
                {kern::TileKind::kForceC2RRows, t.c2r_rows, "c2r_rows"}};
  for (const auto& f : fields)
    if (!kern::tile_ok(f.kind, n, f.w))
      return fail(LPC_ERR_INVALID_ARG, "%s = %d is not an instantiated tile width that fits mesh size %d", f.name, f.w,
                  n);
  return LPC_OK;
}

lpc_status check_cosmo(const lpc_cosmology* c) {
  if (!c) return fail(LPC_ERR_INVALID_ARG, "cosmology is NULL");
  if (!(c->omega_m > 0.0 && c->omega_m <= 1.0)) return fail(LPC_ERR_INVALID_ARG, "omega_m must be in (0, 1]");
  if (!(c->h > 0.0) || !(c->sigma8 > 0.0) || !std::isfinite(c->n_s))
    return fail(LPC_ERR_INVALID_ARG, "h and sigma8 must be positive, n_s finite");
  return LPC_OK;
}

host::Cosmo to_host(const lpc_cosmology* c) { return host::Cosmo{c->omega_m, c->h, c->sigma8, c->n_s}; }

// Reads the device flags (the one synchronisation of a call) and turns them into a status.
lpc_status finish(int* flags, hipStream_t s) {
  int h[kern::kNumFlags] = {0, 0};
  check(hipMemcpyAsync(h, flags, sizeof(h), hipMemcpyDeviceToHost, s), "hipMemcpyAsync(flags)");
  check(hipStreamSynchronize(s), "hipStreamSynchronize");
  g_prof.collect();
  if (h[kern::kFlagNonfinite]) return fail(LPC_ERR_NONFINITE, "a particle coordinate is not finite or far outside the box");
  if (h[kern::kFlagOverflow]) return fail(LPC_ERR_FIXED_OVERFLOW, "a density cell reached 2^63 (more than 32767 particles)");
  return LPC_OK;
}


char* at(void* ws, size_t off) { return static_cast<char*>(ws) + off; }

// ---------------------------------------------------------------------------------------------------------------
// Job tables. A call collects the jobs of every launch it will make into one host buffer, uploads it once into the
// workspace's job region (stream ordered), and then launches with device pointers into that region.
struct Section {
  size_t jobs_off = 0, offs_off = 0;
  int njob = 0, total = 0;
};

// exp(-2 pi i num / den) rounded to FP32 (num / den reduced exactly to [0, 1) first).
float2 unit_root(int64_t num, int64_t den) {
  int64_t r = num % den;
  if (r < 0) r += den;
  const double a = 2.0 * M_PI * static_cast<double>(r) / static_cast<double>(den);
  return make_float2(static_cast<float>(std::cos(a)), static_cast<float>(-std::sin(a)));
}

// The job tables and FFT tables of one call, built on the host and uploaded in one copy to the workspace's job
// region at `dev`.
class JobPack {
 public:
  explicit JobPack(char* dev) : dev_(dev) {}
  // Append `jobs` with `items[i]` work items each (rounded up to multiples of 8); returns the section handle.
  template <class J>
  Section add(const std::vector<J>& jobs, const std::vector<int>& items) {
    Section s;
    s.njob = static_cast<int>(jobs.size());
    std::vector<int> offs(jobs.size() + 1, 0);
    for (size_t i = 0; i < jobs.size(); ++i) offs[i + 1] = offs[i] + round8(items[i]);
    s.total = offs.back();
    s.jobs_off = append(jobs.data(), jobs.size() * sizeof(J));
    s.offs_off = append(offs.data(), offs.size() * sizeof(int));
    return s;
  }
  template <class J>
  Section add1(const J& job, int items) {
    return add(std::vector<J>{job}, std::vector<int>{items});
  }
  size_t bytes() const { return host_.size(); }
  void upload(hipStream_t s) {
    if (host_.size() > kJobRegion) throw HipError{hipErrorInvalidValue, "job tables exceed the workspace job region"};
    check(hipMemcpyAsync(dev_, host_.data(), host_.size(), hipMemcpyHostToDevice, s), "upload job tables");
  }
  // Stage twiddles of plan pl (Plan1D layout, pl.n entries): W_{pR}^{r k} at tw_off[s] + k (R - 1) + r - 1.
  const float2* twiddles(const Plan1D& pl) {
    // keyed by the radix sequence as well: two plans of one length may differ
    int64_t key = pl.n;
    for (int st = 0; st < pl.nst; ++st) key = key * 16 + pl.radix[st];
    auto it = tw_.find(key);
    if (it == tw_.end()) {
      std::vector<float2> t(static_cast<size_t>(pl.n), make_float2(1.f, 0.f));
      for (int st = 0; st < pl.nst; ++st) {
        const int R = pl.radix[st], p = pl.p[st];
        for (int k = 0; k < p; ++k)
          for (int r = 1; r < R; ++r)
            t[static_cast<size_t>(pl.tw_off[st] + k * (R - 1) + r - 1)] =
                unit_root(static_cast<int64_t>(r) * k, static_cast<int64_t>(p) * R);
      }
      it = tw_.emplace(key, append(t.data(), t.size() * sizeof(float2))).first;
    }
    return reinterpret_cast<const float2*>(dev_ + it->second);
  }
  // exp(-2 pi i k / n) for k <= n / 2
  const float2* half_roots(int n) {
    auto it = roots_.find(n);
    if (it == roots_.end()) {
      std::vector<float2> t(static_cast<size_t>(n / 2 + 1));
      for (int k = 0; k <= n / 2; ++k) t[static_cast<size_t>(k)] = unit_root(k, n);
      it = roots_.emplace(n, append(t.data(), t.size() * sizeof(float2))).first;
    }
    return reinterpret_cast<const float2*>(dev_ + it->second);
  }
  // sinc^2(pi m / n) for m <= n / 2 (the CIC window along one axis)
  const float* sinc2(int n) {
    auto it = win_.find(n);
    if (it == win_.end()) {
      std::vector<float> t(static_cast<size_t>(n / 2 + 1), 1.f);
      for (int m = 1; m <= n / 2; ++m) {
        const double x = M_PI * static_cast<double>(m) / n;
        const double v = std::sin(x) / x;
        t[static_cast<size_t>(m)] = static_cast<float>(v * v);
      }
      it = win_.emplace(n, append(t.data(), t.size() * sizeof(float))).first;
    }
    return reinterpret_cast<const float*>(dev_ + it->second);
  }
  // Device copy of n bytes of host data (uploaded with the tables).
  const void* data(const void* p, size_t n) { return dev_ + append(p, n); }
  template <class J>
  const J* jobs(const Section& s) const {
    return reinterpret_cast<const J*>(dev_ + s.jobs_off);
  }
  kern::WorkTable table(const Section& s) const {
    return kern::WorkTable{reinterpret_cast<const int*>(dev_ + s.offs_off), s.njob, s.total};
  }

 private:
  size_t append(const void* p, size_t n) {
    const size_t at = (host_.size() + 63) / 64 * 64;
    host_.resize(at + n);
    std::memcpy(host_.data() + at, p, n);
    return at;
  }
  std::vector<char> host_;
  char* dev_;
  std::map<int64_t, size_t> tw_;
  std::map<int, size_t> roots_, win_;
};

Plan1D plan_of(int n, bool radix12 = true) {
  Plan1D p;
  if (!kern::make_plan(n, &p, radix12)) throw HipError{hipErrorInvalidValue, "unsupported FFT length"};
  return p;
}

// The plan of the force's y passes: 8 x 8 x 12 runs in reverse order, 12 x 8 x 8. On 8-column tiles its radix-12
// stage has one butterfly per thread, so as the first stage it spreads the column loads evenly over the waves (a
// radix-8 stage gives half the waves two butterflies and half one). Measured at 768^3: inverse y 2.33 -> 2.26 ms,
// forward y 0.792 -> 0.786 ms.
Plan1D y_plan_of(int n) {
  const Plan1D p = plan_of(n);
  const bool r12_last = p.nst == 3 && p.radix[0] == 8 && p.radix[1] == 8 && p.radix[2] == 12;
  return r12_last ? kern::reversed_plan(p) : p;
}

// One 3-D transform on an n^3 mesh: the jobs of its passes.
struct R2CSections {
  Section z, y, x;
  int Bz, Pz, Bax, Pax;
  size_t lds_z, lds_ax;
};
struct C2RSections {
  Section x, y, z;
  int Bax, R, Pax;
  size_t lds_ax, lds_z;
};

kern::AxisJob axis_job(JobPack& jp, float2* base, int n, int64_t astr, int64_t ostr, int64_t cstr, int B) {
  kern::AxisJob a{};
  a.base = base;
  a.astr = astr;
  a.ostr = ostr;
  a.cstr = cstr;
  a.n = n;
  a.ncols = n / 2 + 1;
  a.ntc = (a.ncols + B - 1) / B;
  a.per_comp = round8(n * a.ntc);
  a.pl = plan_of(n);
  a.tw = jp.twiddles(a.pl);
  return a;
}

// forward r2c of a real FP32 mesh (fixed = false) or of int64 counts (fixed = true, delta = C mscale - 1)
R2CSections add_r2c(JobPack& jp, const void* in, bool fixed, double mscale, int n, float2* out) {
  R2CSections r;
  const int pitch = kern::mesh_pitch(n);
  const lpc_fft_tiling t = tiling_of(n);
  r.Bz = t.z_rows;
  r.Bax = t.axis_cols;
  r.Pax = kern::axis_points(n, r.Bax);
  r.Pz = kern::r2c_points(n, r.Bz);
  r.lds_z = kern::lds_z_r2c(n, r.Bz);
  r.lds_ax = kern::lds_axis(n, r.Bax);
  kern::ZR2CJob z{};
  z.in = in;
  z.out = out;
  z.mscale = mscale;
  z.n = n;
  z.nrows = n * n;
  z.pitch = pitch;
  z.pl = plan_of(n / 2);
  z.tw = jp.twiddles(z.pl);
  z.roots = jp.half_roots(n);
  r.z = jp.add1(z, (z.nrows + r.Bz - 1) / r.Bz);
  kern::AxisJob y = axis_job(jp, out, n, pitch, static_cast<int64_t>(n) * pitch, 0, r.Bax);
  r.y = jp.add1(y, y.per_comp);
  kern::AxisJob x = axis_job(jp, out, n, static_cast<int64_t>(n) * pitch, pitch, 0, r.Bax);
  r.x = jp.add1(x, x.per_comp);
  (void)fixed;
  return r;
}

C2RSections add_c2r(JobPack& jp, float2* spec, int n, float* out, float scale) {
  C2RSections c;
  const int pitch = kern::mesh_pitch(n);
  const lpc_fft_tiling t = tiling_of(n);
  c.Bax = t.axis_cols;
  c.R = t.z_rows;
  c.Pax = kern::axis_points(n, c.Bax);
  c.lds_ax = kern::lds_axis(n, c.Bax);
  c.lds_z = kern::lds_z_c2r(n, c.R);
  kern::AxisJob x = axis_job(jp, spec, n, static_cast<int64_t>(n) * pitch, pitch, 0, c.Bax);
  c.x = jp.add1(x, x.per_comp);
  kern::AxisJob y = axis_job(jp, spec, n, pitch, static_cast<int64_t>(n) * pitch, 0, c.Bax);
  c.y = jp.add1(y, y.per_comp);
  kern::ZC2RJob z{};
  z.in0 = z.in1 = z.in2 = spec;
  z.out = out;
  z.n = n;
  z.nrows = n * n;
  z.pitch = pitch;
  z.scale = scale;
  z.pl = plan_of(n / 2);
  z.tw = jp.twiddles(z.pl);
  z.roots = jp.half_roots(n);
  c.z = jp.add1(z, (z.nrows + c.R - 1) / c.R);
  return c;
}

void run_r2c(const JobPack& jp, const R2CSections& r, bool fixed, int* flags, hipStream_t s) {
  stage("fft z r2c", s, [&] {
    return kern::launch_z_r2c(jp.jobs<kern::ZR2CJob>(r.z), jp.table(r.z), fixed, r.Bz, r.Pz, r.lds_z, flags, s);
  });
  stage("fft y", s, [&] { return kern::launch_axis(jp.jobs<kern::AxisJob>(r.y), jp.table(r.y), false, r.Bax, r.Pax, r.lds_ax, s); });
  stage("fft x", s, [&] { return kern::launch_axis(jp.jobs<kern::AxisJob>(r.x), jp.table(r.x), false, r.Bax, r.Pax, r.lds_ax, s); });
}

void run_c2r(const JobPack& jp, const C2RSections& c, hipStream_t s) {
  stage("fft x inv", s, [&] { return kern::launch_axis(jp.jobs<kern::AxisJob>(c.x), jp.table(c.x), true, c.Bax, c.Pax, c.lds_ax, s); });
  stage("fft y inv", s, [&] { return kern::launch_axis(jp.jobs<kern::AxisJob>(c.y), jp.table(c.y), true, c.Bax, c.Pax, c.lds_ax, s); });
  stage("fft z c2r", s, [&] { return kern::launch_z_c2r(jp.jobs<kern::ZC2RJob>(c.z), jp.table(c.z), 1, c.R, 0, c.lds_z, s); });
}

// ---------------------------------------------------------------------------------------------------------------
// The PM force of a batch of boxes: every stage is one launch over all boxes.
struct ForceBox {
  int nm;
  double box;
  int64_t n;
  float* pos;         // caller's arrays
  float* vel;
  const float* psi1;
  const float* psi2;
  float* grad;        // pm_force output (or NULL)
  uint64_t* dens;     // int64 counts (written only when the caller asks for them)
  bool keep_counts;   // the caller asked for the int64 counts
  float2 *A, *B, *C;  // three half-spectrum meshes (contiguous: B = A + stride, C = B + stride)
  float* force;       // AoS float3 force mesh
};

struct ForceProgram {
  // sorting: user -> copy 0; copy c -> copy 1 - c; per-copy particle stages
  Section sort_user, sort_next[2], dep[2], parts[2], frame[2], unsort[2];
  Section zr2c, yfwd, pois, yinv, zc2r;
  int Bz = 32, Bax = 32, Bp = 16, R3 = 16;
  int Mp = 8;  // points per thread of the fused x + Poisson tiles: the largest over the boxes
  bool chain_p = false;  // the fused x pass chains its transforms through registers (every plan 8 x 8 x R, 8 columns)
  int P3 = 8;  // points per thread of the three-spectrum c2r tiles: the largest over the boxes
  int Pax = 8;  // points per thread of the strided y tiles: the largest over the boxes
  int Pz = 8;   // points per thread of the forward z tiles: the largest over the boxes
  size_t lds_z = 0, lds_ax = 0, lds_p = 0, lds_c = 0;
  SortSpace ss;
  bool cola_run = false;
  bool fixed_in = false;  // the deposit writes int64 counts for the forward transform (else the FP32 contrast)
};

ForceProgram add_force(JobPack& jp, const std::vector<ForceBox>& boxes, const SortSpace& ss, int deconv,
                       bool cola_run) {
  ForceProgram f;
  f.ss = ss;
  f.cola_run = cola_run;
  for (const ForceBox& b : boxes) f.fixed_in |= b.keep_counts;
  for (const ForceBox& b : boxes) {
    // widths fit every smaller size too, so the smallest over the boxes fits all of them
    const lpc_fft_tiling t = tiling_of(b.nm);
    f.Bz = std::min(f.Bz, t.z_rows);
    f.Bax = std::min(f.Bax, t.axis_cols);
    f.Bp = std::min(f.Bp, t.poisson_cols);
    f.R3 = std::min(f.R3, t.c2r_rows);
  }
  for (const ForceBox& b : boxes) {
    f.Mp = std::max(f.Mp, kern::poisson_points(b.nm, f.Bp));
    f.P3 = std::max(f.P3, kern::c2r_points(b.nm, f.R3));
    f.Pax = std::max(f.Pax, kern::axis_points(b.nm, f.Bax));
    f.Pz = std::max(f.Pz, kern::r2c_points(b.nm, f.Bz));
  }
  f.chain_p = f.Bp == 8;
  for (const ForceBox& b : boxes) f.chain_p = f.chain_p && kern::poisson_chainable(plan_of(b.nm));
  const int ncopy = cola_run ? 2 : 1;
  std::vector<kern::SortJob> su, sn[2];
  std::vector<kern::DepJob> dj[2];
  std::vector<kern::PartJob> pj[2];
  std::vector<kern::UnsortJob> uj[2];
  std::vector<kern::ZR2CJob> zs;
  std::vector<kern::AxisJob> ys;
  std::vector<kern::YGradJob> yis;
  std::vector<kern::PoissonJob> ps;
  std::vector<kern::ZC2RJob> cs;
  std::vector<int> i_part, i_frame, i_tile, i_z, i_y, i_yi, i_p, i_c;
  for (size_t ib = 0; ib < boxes.size(); ++ib) {
    const ForceBox& b = boxes[ib];
    const int nm = b.nm, pitch = kern::mesh_pitch(nm), nh = nm / 2 + 1;
    const int64_t M = static_cast<int64_t>(nm) * nm * nm;
    const double scale = (static_cast<double>(nm) * 65536.0) / b.box;
    const kern::TileGrid nt = ss.nt[ib];
    i_part.push_back(static_cast<int>((b.n + kern::kNT - 1) / kern::kNT));
    i_frame.push_back(static_cast<int>((3 * b.n + kern::kNT - 1) / kern::kNT));
    i_tile.push_back(nt.count());
    auto sort_job = [&](const BoxParts* src, const BoxParts& dst) {
      kern::SortJob j{};
      if (src) {
        j.pos = src->pos;
        j.vel = src->vel;
        j.psi1 = src->psi1;
        j.psi2 = src->psi2;
        j.orig = src->orig;
      } else {
        j.pos = b.pos;
        j.vel = b.vel;
        j.psi1 = b.psi1;
        j.psi2 = b.psi2;
      }
      j.dpos = dst.pos;
      j.dvel = dst.vel;
      j.dpsi1 = (j.psi1 && j.psi2) ? dst.psi1 : nullptr;  // a plain PM run may pass no displacements
      j.dpsi2 = (j.psi1 && j.psi2) ? dst.psi2 : nullptr;
      j.dorig = dst.orig;
      j.n = b.n;
      j.pbase = ss.pbase[ib];
      j.tbase = ss.tbase[ib];
      j.ntx = nt.x;
      j.nty = nt.y;
      j.ntz = nt.z;
      j.nm = nm;
      j.scale = scale;
      return j;
    };
    su.push_back(sort_job(nullptr, ss.copy[0][ib]));
    for (int c = 0; c < ncopy; ++c) {
      const BoxParts& cp = ss.copy[c][ib];
      if (cola_run) sn[c].push_back(sort_job(&cp, ss.copy[1 - c][ib]));
      kern::DepJob d{};
      d.pos = cp.pos;
      d.n = b.n;
      d.pbase = ss.pbase[ib];
      d.tbase = ss.tbase[ib];
      d.ntx = nt.x;
      d.nty = nt.y;
      d.ntz = nt.z;
      d.inv_yz = kern::div_inverse(nt.y * nt.z);
      d.inv_z = kern::div_inverse(nt.z);
      d.nm = nm;
      d.scale = scale;
      d.mscale = (static_cast<double>(M) / static_cast<double>(b.n)) * 0x1.0p-48;
      d.dens = f.fixed_in ? b.dens : nullptr;
      d.delta = f.fixed_in ? nullptr : b.force;  // the contrast takes the start of the density / force region
      dj[c].push_back(d);
      kern::PartJob p{};
      p.pos = cp.pos;
      p.vel = cp.vel;
      p.psi1 = cp.psi1;
      p.psi2 = cp.psi2;
      p.n = b.n;
      p.force = b.force;
      p.grad = b.grad;
      p.orig = cp.orig;
      p.nm = nm;
      p.box = static_cast<float>(b.box);
      p.scale = scale;
      p.pbase = ss.pbase[ib];
      p.tbase = ss.tbase[ib];
      p.ntx = nt.x;
      p.nty = nt.y;
      p.ntz = nt.z;
      pj[c].push_back(p);
      kern::UnsortJob u{};
      u.spos = cp.pos;
      u.svel = cp.vel;
      u.orig = cp.orig;
      u.pos = b.pos;
      u.vel = b.vel;
      u.n = b.n;
      uj[c].push_back(u);
    }
    kern::ZR2CJob z{};
    z.in = f.fixed_in ? static_cast<const void*>(b.dens) : static_cast<const void*>(b.force);
    z.out = b.A;
    z.mscale = (static_cast<double>(M) / static_cast<double>(b.n)) * 0x1.0p-48;
    z.n = nm;
    z.nrows = nm * nm;
    z.pitch = pitch;
    z.pl = plan_of(nm / 2);
    z.tw = jp.twiddles(z.pl);
    z.roots = jp.half_roots(nm);
    zs.push_back(z);
    i_z.push_back((z.nrows + f.Bz - 1) / f.Bz);
    kern::AxisJob y = axis_job(jp, b.A, nm, pitch, static_cast<int64_t>(nm) * pitch, 0, f.Bax);
    y.pl = y_plan_of(nm);
    y.tw = jp.twiddles(y.pl);
    ys.push_back(y);
    i_y.push_back(y.per_comp);
    kern::YGradJob yi{};
    yi.A = b.A;
    yi.B = b.B;
    yi.C = b.C;
    yi.astr = pitch;
    yi.ostr = static_cast<int64_t>(nm) * pitch;
    yi.n = nm;
    yi.ncols = nh;
    yi.ntc = (nh + f.Bax - 1) / f.Bax;
    yi.per_comp = round8(nm * yi.ntc);
    yi.ntc1 = (nh + f.Bax / 2 - 1) / (f.Bax / 2);
    yi.per_comp1 = round8(nm * yi.ntc1);
    yi.kf = static_cast<float>(2.0 * M_PI / b.box);
    yi.pl = y_plan_of(nm);
    yi.tw = jp.twiddles(yi.pl);
    yis.push_back(yi);
    i_yi.push_back(yi.per_comp + yi.per_comp1);  // component 0: the x gradient; 1: the potential (y and z gradients)
    kern::PoissonJob p{};
    p.A = b.A;
    p.B = b.B;
    p.C = b.C;
    p.nm = nm;
    p.pitch = pitch;
    p.ntc = (nh + f.Bp - 1) / f.Bp;
    p.deconv = deconv;
    p.kf = static_cast<float>(2.0 * M_PI / b.box);
    p.inv_m3 = static_cast<float>(1.0 / static_cast<double>(M));
    p.pl = plan_of(nm);
    p.tw = jp.twiddles(p.pl);
    p.tw_rev = jp.twiddles(kern::reversed_plan(p.pl));
    p.win = jp.sinc2(nm);
    ps.push_back(p);
    i_p.push_back(nm * p.ntc);
    kern::ZC2RJob c{};
    c.in0 = b.A;
    c.in1 = b.B;
    c.in2 = b.C;
    c.out = b.force;
    c.n = nm;
    c.nrows = nm * nm;
    c.pitch = pitch;
    c.scale = 1.0f;
    c.kz3 = static_cast<float>(2.0 * M_PI / b.box);  // C holds the potential: i k_z applied on load
    // this pass sits at its register cap (six waves per SIMD); the radix-12 stage would push it into scratch
    c.pl = plan_of(nm / 2, false);
    c.tw = jp.twiddles(c.pl);
    c.roots = jp.half_roots(nm);
    cs.push_back(c);
    i_c.push_back((c.nrows + f.R3 - 1) / f.R3);
    f.lds_z = std::max(f.lds_z, kern::lds_z_r2c(nm, f.Bz));
    f.lds_ax = std::max(f.lds_ax, kern::lds_axis(nm, f.Bax));
    f.lds_p = std::max(f.lds_p, kern::lds_x_poisson(nm, f.Bp, f.Mp, f.chain_p));
    f.lds_c = std::max(f.lds_c, kern::lds_z_c2r(nm, 3 * f.R3));
  }
  f.sort_user = jp.add(su, i_part);
  for (int c = 0; c < ncopy; ++c) {
    if (cola_run) f.sort_next[c] = jp.add(sn[c], i_part);
    f.dep[c] = jp.add(dj[c], i_tile);
    f.parts[c] = jp.add(pj[c], i_part);
    f.frame[c] = jp.add(pj[c], i_frame);
    f.unsort[c] = jp.add(uj[c], i_part);
  }
  f.zr2c = jp.add(zs, i_z);
  f.yfwd = jp.add(ys, i_y);
  f.pois = jp.add(ps, i_p);
  f.yinv = jp.add(yis, i_yi);
  f.zc2r = jp.add(cs, i_c);
  return f;
}

// Tile sort of every box (counts cleared by a kernel, so the sequence may be recorded in a graph).
// keys_done: the key pass already ran (folded into the previous drift), so only the scan and the scatter remain
void run_sort(const JobPack& jp, const SortSpace& ss, const Section& sec, int* flags, hipStream_t s,
              bool keys_done = false) {
  if (!keys_done) {
    stage("sort keys", s, [&] { return kern::fill_i32(ss.cnt, static_cast<size_t>(ss.G), 0, s); });
    stage("sort keys", s, [&] {
      return kern::launch_tile_key(jp.jobs<kern::SortJob>(sec), jp.table(sec), ss.cnt, ss.key, ss.rank, flags, s);
    });
  }
  stage("sort scan", s, [&] { return kern::launch_scan(ss.cnt, ss.start, ss.G, ss.block_sums, s); });
  stage("sort scatter", s, [&] {
    return kern::launch_scatter(jp.jobs<kern::SortJob>(sec), jp.table(sec), ss.key, ss.rank, ss.start, s);
  });
}

// deposit (from sorted copy c) -> delta -> forward FFT -> Poisson/gradient -> inverse FFTs -> AoS force meshes
void run_force_mesh(const JobPack& jp, const ForceProgram& f, int c, int* flags, hipStream_t s) {
  stage("deposit", s, [&] {
    return kern::launch_deposit_tiles(jp.jobs<kern::DepJob>(f.dep[c]), jp.table(f.dep[c]), f.ss.start, flags, s);
  });
  stage("fft z r2c", s, [&] {
    return kern::launch_z_r2c(jp.jobs<kern::ZR2CJob>(f.zr2c), jp.table(f.zr2c), f.fixed_in, f.Bz, f.Pz, f.lds_z, flags,
                              s);
  });
  stage("fft y", s, [&] { return kern::launch_axis(jp.jobs<kern::AxisJob>(f.yfwd), jp.table(f.yfwd), false, f.Bax, f.Pax, f.lds_ax, s); });
  stage("fft x + poisson", s, [&] { return kern::launch_poisson(jp.jobs<kern::PoissonJob>(f.pois), jp.table(f.pois), f.Bp, f.Mp, f.chain_p, f.lds_p, s); });
  stage("fft y inv", s, [&] { return kern::launch_y_grad(jp.jobs<kern::YGradJob>(f.yinv), jp.table(f.yinv), f.Bax, f.Pax, f.lds_ax, s); });
  stage("fft z c2r", s, [&] { return kern::launch_z_c2r(jp.jobs<kern::ZC2RJob>(f.zc2r), jp.table(f.zc2r), 3, f.R3, f.P3, f.lds_c, s); });
}

// The whole COLA run over a_list for every box (all boxes share cosmology, stepping and time list). Particles are
// tile-sorted into workspace copy 0 first, re-sorted into the other copy before every later force evaluation, and
// copied back to the caller's order at the end.
// lc (optional): per drift i, the lightcone step (active when its table pointer is set).
void run_cola(const JobPack& jp, const ForceProgram& f, const std::vector<double>& tab, int n_a, double om, bool cola,
              int* flags, hipStream_t s, const std::vector<kern::LightconeStep>* lc = nullptr) {
  auto row = [&tab](int i) { return tab.data() + static_cast<size_t>(i) * host::kCoefColumns; };
  int c = 0;
  run_sort(jp, f.ss, f.sort_user, flags, s);
  if (cola) {
    const float f1 = static_cast<float>(-row(0)[host::kF1]), f2 = static_cast<float>(-row(0)[host::kF2]);
    stage("frame velocity", s, [&] { return kern::launch_frame(jp.jobs<kern::PartJob>(f.frame[c]), jp.table(f.frame[c]), f1, f2, s); });
  }
  for (int i = 0; i < n_a; ++i) {
    if (i > 0) {
      run_sort(jp, f.ss, f.sort_next[c], flags, s, true);
      c = 1 - c;
    }
    const double* r = row(i);
    run_force_mesh(jp, f, c, flags, s);
    kern::KickDrift kd;
    kd.kick = static_cast<float>(r[host::kK] * (-1.5 * om));
    kd.d1 = static_cast<float>(r[host::kD1]);
    kd.d2m = static_cast<float>(r[host::kD2] - r[host::kD1] * r[host::kD1]);
    kd.drift = static_cast<float>(r[host::kQ]);
    kd.dd1 = static_cast<float>(r[host::kDD1]);
    kd.dd2 = static_cast<float>(r[host::kDD2]);
    kd.do_drift = (i + 1 < n_a) ? 1 : 0;
    kd.cola = cola ? 1 : 0;
    // a drift is followed by a re-sort: its key pass runs inside this kernel, on zeroed bucket counts
    const bool keys = kd.do_drift != 0;
    if (keys) stage("sort keys", s, [&] { return kern::fill_i32(f.ss.cnt, static_cast<size_t>(f.ss.G), 0, s); });
    if (lc && kd.do_drift && (*lc)[static_cast<size_t>(i)].tab) {
      stage("gather kick drift lightcone", s, [&] {
        return kern::launch_gather_kick_drift_lc(jp.jobs<kern::PartJob>(f.parts[c]), jp.table(f.parts[c]), kd,
                                                 (*lc)[static_cast<size_t>(i)], flags, f.ss.cnt, f.ss.key, f.ss.rank,
                                                 s);
      });
      continue;
    }
    stage("gather kick drift", s, [&] {
      return kern::launch_gather_kick_drift(jp.jobs<kern::PartJob>(f.parts[c]), jp.table(f.parts[c]), kd, flags,
                                            keys ? f.ss.cnt : nullptr, keys ? f.ss.key : nullptr,
                                            keys ? f.ss.rank : nullptr, s);
    });
  }
  if (cola) {
    const double* r = row(n_a - 1);
    const float f1 = static_cast<float>(r[host::kF1]), f2 = static_cast<float>(r[host::kF2]);
    stage("frame velocity", s, [&] { return kern::launch_frame(jp.jobs<kern::PartJob>(f.frame[c]), jp.table(f.frame[c]), f1, f2, s); });
  }
  stage("unsort", s, [&] { return kern::launch_unsort(jp.jobs<kern::UnsortJob>(f.unsort[c]), jp.table(f.unsort[c]), s); });
}

ForceBox force_box(void* ws, const Plan& p, int nm, double box, int64_t n, float* pos, float* vel, const float* psi1,
                   const float* psi2, float* grad, uint64_t* dens_override) {
  ForceBox b{};
  b.nm = nm;
  b.box = box;
  b.n = n;
  b.pos = pos;
  b.vel = vel;
  b.psi1 = psi1;
  b.psi2 = psi2;
  b.grad = grad;
  b.dens = dens_override ? dens_override : reinterpret_cast<uint64_t*>(at(ws, p.dens));
  b.keep_counts = dens_override != nullptr;
  b.A = reinterpret_cast<float2*>(at(ws, p.A));
  b.B = reinterpret_cast<float2*>(at(ws, p.B));
  b.C = reinterpret_cast<float2*>(at(ws, p.C));
  b.force = reinterpret_cast<float*>(at(ws, p.dens));
  return b;
}

lpc_status check_geom_mesh(const lpc_geometry* g) {
  if (!g) return fail(LPC_ERR_INVALID_ARG, "geometry is NULL");
  if (!(g->box > 0.0) || !std::isfinite(g->box)) return fail(LPC_ERR_INVALID_ARG, "box must be positive");
  return check_mesh(g->n_mesh, "n_mesh");
}

lpc_status check_particles(const lpc_particles* p, bool need_psi) {
  if (!p) return fail(LPC_ERR_INVALID_ARG, "particles is NULL");
  if (p->n < 0) return fail(LPC_ERR_INVALID_ARG, "n < 0");
  if (p->n > 0 && (!p->pos || !p->vel)) return fail(LPC_ERR_INVALID_ARG, "pos/vel is NULL");
  if (p->n > 0 && need_psi && (!p->psi1 || !p->psi2)) return fail(LPC_ERR_INVALID_ARG, "psi1/psi2 is NULL");
  if (p->n > (int64_t(1) << 31) - 1) return fail(LPC_ERR_INVALID_ARG, "n exceeds 2^31 - 1");
  return LPC_OK;
}

lpc_status check_stepping(const lpc_stepping* step) {
  if (!step) return fail(LPC_ERR_INVALID_ARG, "stepping is NULL");
  if (step->deconv_power < 0 || step->deconv_power > 2) return fail(LPC_ERR_INVALID_ARG, "deconv_power not in 0..2");
  if (step->reserved != 0) return fail(LPC_ERR_INVALID_ARG, "stepping.reserved must be 0");
  return LPC_OK;
}

// Argument checks of lpc_pm_force and lpc_pm_force_noalloc (nothing is enqueued when they fail).
lpc_status check_pm_force_args(const lpc_geometry* geom, const lpc_stepping* step, const float* pos, int64_t n,
                               const float* grad_out) {
  if (lpc_status st = check_geom_mesh(geom)) return st;
  if (!step) return fail(LPC_ERR_INVALID_ARG, "stepping is NULL");
  if (step->deconv_power < 0 || step->deconv_power > 2) return fail(LPC_ERR_INVALID_ARG, "deconv_power not in 0..2");
  if (n <= 0 || n > (int64_t(1) << 31) - 1) return fail(LPC_ERR_INVALID_ARG, "n must be in [1, 2^31 - 1]");
  if (!pos || !grad_out) return fail(LPC_ERR_INVALID_ARG, "pos/grad_out is NULL");
  return LPC_OK;
}

// The PM force of one box on workspace ws (arguments already checked).
lpc_status pm_force_impl(const lpc_geometry* geom, const lpc_stepping* step, const float* pos, int64_t n,
                         float* grad_out, int64_t* density_fixed_out, void* ws, size_t ws_bytes, void* stream) {
  const Plan p = make_ws_plan(geom->n_mesh, LPC_OP_PM_FORCE, n);
  if (lpc_status st = check_ws(ws, ws_bytes, p.total)) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  return guarded([&]() {
    int* flags = reinterpret_cast<int*>(ws);
    stage("clear flags", s, [&] { return kern::fill_i32(flags, kern::kNumFlags, 0, s); });
    JobPack jp(at(ws, p.jobs));
    const ForceBox b = force_box(ws, p, geom->n_mesh, geom->box, n, const_cast<float*>(pos), nullptr, nullptr, nullptr,
                                 grad_out, reinterpret_cast<uint64_t*>(density_fixed_out));
    const ForceProgram f = add_force(jp, {b}, sort_space(ws, p, geom->n_mesh, LPC_OP_PM_FORCE, n), step->deconv_power,
                                     false);
    jp.upload(s);
    run_sort(jp, f.ss, f.sort_user, flags, s);
    run_force_mesh(jp, f, 0, flags, s);
    stage("gather", s, [&] { return kern::launch_gather(jp.jobs<kern::PartJob>(f.parts[0]), jp.table(f.parts[0]), flags, s); });
    return finish(flags, s);
  });
}

// Static scratch of lpc_pm_force_noalloc: device memory that the library never allocates at run time. Each GPU
// holds its own copy from the library's load until the process ends; host code reaches it only through the address
// hipGetSymbolAddress returns for the current device (the array's name in host code is not a device address).
constexpr size_t kScratchBytes = LPC_NOALLOC_SCRATCH_BYTES;
__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// The device address of the current device's scratch, looked up once per device.
lpc_status scratch_of_current_device(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
    return fail(LPC_ERR_HIP, "lpc_pm_force_noalloc: no current HIP device (or device index >= %d)", kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(LPC_ERR_HIP, "hipGetSymbolAddress(scratch) on device %d failed: %s", dev, hipGetErrorString(e));
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return LPC_OK;
}

// Cached hipGraph of one batched run: replayed while the call's arguments stay the same.
struct GraphCache {
  std::vector<char> key;
  hipGraphExec_t exec = nullptr;
};
GraphCache g_graph;
bool g_graph_on = true;

// The stream batched runs are captured on (capture only records launches; the graph runs on the caller's stream).
hipStream_t capture_stream() {
  static hipStream_t cs = [] {
    hipStream_t st;
    check(hipStreamCreateWithFlags(&st, hipStreamNonBlocking), "hipStreamCreateWithFlags");
    return st;
  }();
  return cs;
}

}  // namespace

extern "C" {

size_t lpc_workspace_bytes(const lpc_geometry* geom, int32_t op, int64_t n_particles) {
  if (!geom) return 0;
  const int n = (op == LPC_OP_INIT_IC) ? geom->n_side : geom->n_mesh;
  if (!fft_size_ok(n)) return 0;
  const bool takes_particles = (op == LPC_OP_PM_FORCE || op == LPC_OP_COLA_STEP || op == LPC_OP_POWER_SPECTRUM ||
                                op == LPC_OP_BISPECTRUM);
  if (takes_particles && (n_particles < 1 || n_particles > (int64_t(1) << 31) - 1)) return 0;
  return make_ws_plan(n, op, n_particles).total;
}

int32_t lpc_fft_pitch(int32_t n) { return (n >= 2) ? kern::mesh_pitch(n) : 0; }

lpc_status lpc_fft_tiling_default(int32_t n_mesh, lpc_fft_tiling* out) {
  if (lpc_status st = check_mesh(n_mesh, "n_mesh")) return st;
  if (!out) return fail(LPC_ERR_INVALID_ARG, "out is NULL");
  *out = default_tiling(n_mesh);
  return LPC_OK;
}

lpc_status lpc_fft_tiling_get(int32_t n_mesh, lpc_fft_tiling* out) {
  if (lpc_status st = check_mesh(n_mesh, "n_mesh")) return st;
  if (!out) return fail(LPC_ERR_INVALID_ARG, "out is NULL");
  *out = tiling_of(n_mesh);
  return LPC_OK;
}

lpc_status lpc_fft_tiling_set(int32_t n_mesh, const lpc_fft_tiling* t) {
  if (lpc_status st = check_mesh(n_mesh, "n_mesh")) return st;
  if (t)
    if (lpc_status st = check_tiling(n_mesh, *t)) return st;
  std::lock_guard<std::mutex> lock(g_tiling.mu);
  if (t)
    g_tiling.over[n_mesh] = *t;
  else
    g_tiling.over.erase(n_mesh);
  ++g_tiling.generation;
  return LPC_OK;
}

lpc_status lpc_fft_tiling_reset(void) {
  std::lock_guard<std::mutex> lock(g_tiling.mu);
  g_tiling.over.clear();
  ++g_tiling.generation;
  return LPC_OK;
}

lpc_status lpc_profile_enable(int32_t on) {
  g_prof.on = (on != 0);
  return LPC_OK;
}

lpc_status lpc_profile_reset(void) {
  g_prof.stats.clear();
  return LPC_OK;
}

int32_t lpc_profile_count(void) { return static_cast<int32_t>(g_prof.stats.size()); }

lpc_status lpc_profile_get(int32_t i, const char** name, int64_t* launches, double* total_ms) {
  if (i < 0 || i >= static_cast<int32_t>(g_prof.stats.size()) || !name || !launches || !total_ms)
    return fail(LPC_ERR_INVALID_ARG, "profile index out of range or NULL output");
  const auto& kv = g_prof.stats[static_cast<size_t>(i)];
  *name = kv.first.c_str();
  *launches = kv.second.launches;
  *total_ms = kv.second.total_ms;
  return LPC_OK;
}

const char* lpc_status_string(lpc_status s) {
  switch (s) {
    case LPC_OK: return "LPC_OK";
    case LPC_ERR_INVALID_ARG: return "LPC_ERR_INVALID_ARG";
    case LPC_ERR_UNSUPPORTED_SIZE: return "LPC_ERR_UNSUPPORTED_SIZE";
    case LPC_ERR_WORKSPACE: return "LPC_ERR_WORKSPACE";
    case LPC_ERR_HIP: return "LPC_ERR_HIP";
    case LPC_ERR_FIXED_OVERFLOW: return "LPC_ERR_FIXED_OVERFLOW";
    case LPC_ERR_NONFINITE: return "LPC_ERR_NONFINITE";
    case LPC_ERR_CAPACITY: return "LPC_ERR_CAPACITY";
  }
  return "unknown lpc_status";
}

const char* lpc_last_error(void) { return lpc::abi::last_error(); }

lpc_status lpc_cola_coefficients(const lpc_cosmology* cosmo, const lpc_stepping* step, const double* a_list,
                                 int32_t n_a, double* out) {
  if (lpc_status st = check_cosmo(cosmo)) return st;
  if (!step || !a_list || !out) return fail(LPC_ERR_INVALID_ARG, "NULL argument");
  if (n_a < 2) return fail(LPC_ERR_INVALID_ARG, "need at least two times");
  for (int i = 0; i < n_a; ++i) {
    if (!(a_list[i] > 0.0) || !std::isfinite(a_list[i])) return fail(LPC_ERR_INVALID_ARG, "a_list[%d] not positive", i);
    if (i > 0 && !(a_list[i] > a_list[i - 1])) return fail(LPC_ERR_INVALID_ARG, "a_list not strictly increasing");
  }
  if (step->modified && !(step->n_lpt != 0.0 && std::isfinite(step->n_lpt)))
    return fail(LPC_ERR_INVALID_ARG, "n_lpt must be finite and non-zero");
  return guarded([&]() {
    host::coefficient_table(to_host(cosmo), step->modified != 0, step->n_lpt, a_list, n_a, out);
    return LPC_OK;
  });
}

lpc_status lpc_linear_power(const lpc_cosmology* cosmo, const double* k, int32_t m, double* pk) {
  if (lpc_status st = check_cosmo(cosmo)) return st;
  if (m < 0 || (m > 0 && (!k || !pk))) return fail(LPC_ERR_INVALID_ARG, "bad k/pk arrays");
  return guarded([&]() {
    const host::Cosmo c = to_host(cosmo);
    const double A = host::pk_amplitude(c);
    for (int i = 0; i < m; ++i) pk[i] = host::linear_pk(c, A, k[i]);
    return LPC_OK;
  });
}

lpc_status lpc_pm_force(const lpc_geometry* geom, const lpc_stepping* step, const float* pos, int64_t n,
                        float* grad_out, int64_t* density_fixed_out, void* ws, size_t ws_bytes, void* stream) {
  if (lpc_status st = check_pm_force_args(geom, step, pos, n, grad_out)) return st;
  return pm_force_impl(geom, step, pos, n, grad_out, density_fixed_out, ws, ws_bytes, stream);
}

lpc_status lpc_pm_force_noalloc(const lpc_geometry* geom, const lpc_stepping* step, const float* pos, int64_t n,
                                float* grad_out, int64_t* density_fixed_out, void* stream) {
  if (lpc_status st = check_pm_force_args(geom, step, pos, n, grad_out)) return st;
  const size_t need = make_ws_plan(geom->n_mesh, LPC_OP_PM_FORCE, n).total;
  if (need > kScratchBytes)
    return fail(LPC_ERR_WORKSPACE,
                "lpc_pm_force_noalloc: a %d^3 mesh with %lld particles needs %zu bytes of scratch; the static scratch "
                "holds %zu (LPC_NOALLOC_SCRATCH_BYTES)",
                geom->n_mesh, static_cast<long long>(n), need, kScratchBytes);
  void* ws = nullptr;
  if (lpc_status st = scratch_of_current_device(&ws)) return st;
  return pm_force_impl(geom, step, pos, n, grad_out, density_fixed_out, ws, kScratchBytes, stream);
}

lpc_status lpc_cola_step(const lpc_geometry* geom, const lpc_cosmology* cosmo, const lpc_stepping* step,
                         const double* a_list, int32_t n_a, const lpc_particles* inout, void* ws, size_t ws_bytes,
                         void* stream) {
  if (lpc_status st = check_geom_mesh(geom)) return st;
  if (lpc_status st = check_cosmo(cosmo)) return st;
  if (lpc_status st = check_stepping(step)) return st;
  if (lpc_status st = check_particles(inout, step->cola != 0)) return st;
  if (inout->n == 0) return fail(LPC_ERR_INVALID_ARG, "no particles");
  std::vector<double> tab(static_cast<size_t>(n_a > 0 ? n_a : 0) * host::kCoefColumns);
  if (lpc_status st = lpc_cola_coefficients(cosmo, step, a_list, n_a, tab.data())) return st;
  const Plan p = make_ws_plan(geom->n_mesh, LPC_OP_COLA_STEP, inout->n);
  if (lpc_status st = check_ws(ws, ws_bytes, p.total)) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  return guarded([&]() {
    int* flags = reinterpret_cast<int*>(ws);
    stage("clear flags", s, [&] { return kern::fill_i32(flags, kern::kNumFlags, 0, s); });
    JobPack jp(at(ws, p.jobs));
    const ForceBox b = force_box(ws, p, geom->n_mesh, geom->box, inout->n, inout->pos, inout->vel, inout->psi1,
                                 inout->psi2, nullptr, nullptr);
    const ForceProgram f = add_force(jp, {b}, sort_space(ws, p, geom->n_mesh, LPC_OP_COLA_STEP, inout->n),
                                     step->deconv_power, true);
    jp.upload(s);
    run_cola(jp, f, tab, n_a, cosmo->omega_m, step->cola != 0, flags, s);
    return finish(flags, s);
  });
}

lpc_status lpc_comoving_distance(const lpc_cosmology* cosmo, const double* a, int32_t m, double* r) {
  if (lpc_status st = check_cosmo(cosmo)) return st;
  if (m < 0 || (m > 0 && (!a || !r))) return fail(LPC_ERR_INVALID_ARG, "bad a/r arrays");
  for (int i = 0; i < m; ++i)
    if (!(a[i] > 0.0 && a[i] <= 1.0)) return fail(LPC_ERR_INVALID_ARG, "a[%d] must be in (0, 1]", i);
  return guarded([&]() {
    const host::Cosmo c = to_host(cosmo);
    for (int i = 0; i < m; ++i) r[i] = host::comoving_distance(c, a[i]);
    return LPC_OK;
  });
}

lpc_status lpc_cola_step_lightcone(const lpc_geometry* geom, const lpc_cosmology* cosmo, const lpc_stepping* step,
                                   const double* a_list, int32_t n_a, const lpc_particles* inout,
                                   const lpc_lightcone* lc, int64_t* n_records, void* ws, size_t ws_bytes,
                                   void* stream) {
  if (lpc_status st = check_geom_mesh(geom)) return st;
  if (lpc_status st = check_cosmo(cosmo)) return st;
  if (lpc_status st = check_stepping(step)) return st;
  if (lpc_status st = check_particles(inout, step->cola != 0)) return st;
  if (inout->n == 0) return fail(LPC_ERR_INVALID_ARG, "no particles");
  if (!lc || !n_records) return fail(LPC_ERR_INVALID_ARG, "lightcone or n_records is NULL");
  if (lc->capacity < 0 || (lc->capacity > 0 && !lc->records))
    return fail(LPC_ERR_INVALID_ARG, "lightcone capacity < 0, or records NULL with capacity > 0");
  int64_t nrep = 1;
  for (int d = 0; d < 3; ++d) {
    if (!std::isfinite(lc->origin[d])) return fail(LPC_ERR_INVALID_ARG, "origin not finite");
    if (lc->rep_lo[d] > lc->rep_hi[d]) return fail(LPC_ERR_INVALID_ARG, "rep_lo[%d] > rep_hi[%d]", d, d);
    if (lc->rep_lo[d] < -1024 || lc->rep_hi[d] > 1024) return fail(LPC_ERR_INVALID_ARG, "replicate range beyond +-1024");
    nrep *= static_cast<int64_t>(lc->rep_hi[d]) - lc->rep_lo[d] + 1;
  }
  if (nrep > 32768) return fail(LPC_ERR_INVALID_ARG, "more than 32768 replicates");
  if (!(lc->a_start > 0.0) || !std::isfinite(lc->a_start)) return fail(LPC_ERR_INVALID_ARG, "a_start must be positive");
  if (n_a > 1000) return fail(LPC_ERR_INVALID_ARG, "a lightcone run takes at most 1000 times");
  std::vector<double> tab(static_cast<size_t>(n_a > 0 ? n_a : 0) * host::kCoefColumns);
  if (lpc_status st = lpc_cola_coefficients(cosmo, step, a_list, n_a, tab.data())) return st;
  if (a_list[n_a - 1] > 1.0) return fail(LPC_ERR_INVALID_ARG, "a lightcone run ends at a <= 1");
  const Plan p = make_ws_plan(geom->n_mesh, LPC_OP_COLA_STEP, inout->n);
  if (lpc_status st = check_ws(ws, ws_bytes, p.total)) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  *n_records = 0;
  return guarded([&]() {
    const host::Cosmo c = to_host(cosmo);
    int* flags = reinterpret_cast<int*>(ws);
    // the record counter sits in the flag region (64 bytes in, 8 bytes)
    unsigned long long* counter = reinterpret_cast<unsigned long long*>(at(ws, 64));
    stage("clear flags", s, [&] { return kern::fill_i32(flags, kern::kNumFlags, 0, s); });
    stage("clear flags", s, [&] { return kern::fill_i32(reinterpret_cast<int*>(counter), 2, 0, s); });
    JobPack jp(at(ws, p.jobs));
    const ForceBox b = force_box(ws, p, geom->n_mesh, geom->box, inout->n, inout->pos, inout->vel, inout->psi1,
                                 inout->psi2, nullptr, nullptr);
    const ForceProgram f = add_force(jp, {b}, sort_space(ws, p, geom->n_mesh, LPC_OP_COLA_STEP, inout->n),
                                     step->deconv_power, true);
    // Replicates sorted by their closest distance to the observer: the ones a drift still needs (closest point
    // within R_L(a_i), Sec. 6.2.3) are then a prefix of the list.
    struct Rep {
      double dmin;
      int v[4];
    };
    std::vector<Rep> reps;
    const int ny = lc->rep_hi[1] - lc->rep_lo[1] + 1, nz = lc->rep_hi[2] - lc->rep_lo[2] + 1;
    for (int ix = lc->rep_lo[0]; ix <= lc->rep_hi[0]; ++ix)
      for (int iy = lc->rep_lo[1]; iy <= lc->rep_hi[1]; ++iy)
        for (int iz = lc->rep_lo[2]; iz <= lc->rep_hi[2]; ++iz) {
          const int ijk[3] = {ix, iy, iz};
          double d2 = 0.0;
          for (int d = 0; d < 3; ++d) {
            const double lo = ijk[d] * geom->box, hi = lo + geom->box, o = lc->origin[d];
            const double e = std::max(0.0, std::max(lo - o, o - hi));
            d2 += e * e;
          }
          const int flat = ((ix - lc->rep_lo[0]) * ny + (iy - lc->rep_lo[1])) * nz + (iz - lc->rep_lo[2]);
          reps.push_back(Rep{std::sqrt(d2), {ix, iy, iz, flat}});
        }
    std::stable_sort(reps.begin(), reps.end(), [](const Rep& x, const Rep& y) { return x.dmin < y.dmin; });
    std::vector<int> rep_ints;
    for (const Rep& r : reps) rep_ints.insert(rep_ints.end(), r.v, r.v + 4);
    const int* reps_dev = static_cast<const int*>(jp.data(rep_ints.data(), rep_ints.size() * sizeof(int)));
    const bool modified = step->modified != 0, cola = step->cola != 0;
    std::vector<kern::LightconeStep> lcs(static_cast<size_t>(n_a));
    for (int i = 0; i + 1 < n_a; ++i) {
      const double ai = a_list[i], an = a_list[i + 1];
      if (ai < lc->a_start) continue;
      kern::LightconeStep& L = lcs[static_cast<size_t>(i)];
      const double rli = host::comoving_distance(c, ai), rln = host::comoving_distance(c, an);
      int nact = 0;
      while (nact < static_cast<int>(reps.size()) && reps[static_cast<size_t>(nact)].dmin <= rli) ++nact;
      // partial drift from a_i to a = a_i + t (a_{i+1} - a_i) at t = k / (kLcTab - 1)
      std::vector<float> tb(3 * kern::kLcTab);
      const double d1i = host::growth_D1(c, ai), d2i = host::growth_D2(c, ai);
      for (int k = 0; k < kern::kLcTab; ++k) {
        const double a = (k == kern::kLcTab - 1) ? an : ai + (an - ai) * k / (kern::kLcTab - 1.0);
        tb[3 * k] = static_cast<float>(host::partial_drift_factor(c, ai, a, an, modified, step->n_lpt));
        tb[3 * k + 1] = static_cast<float>(host::growth_D1(c, a) - d1i);
        tb[3 * k + 2] = static_cast<float>(host::growth_D2(c, a) - d2i);
      }
      L.ai = static_cast<float>(ai);
      L.aip1 = static_cast<float>(an);
      L.rli = static_cast<float>(rli);
      L.rln = static_cast<float>(rln);
      L.ox = static_cast<float>(lc->origin[0]);
      L.oy = static_cast<float>(lc->origin[1]);
      L.oz = static_cast<float>(lc->origin[2]);
      if (cola) {
        const double am = 0.5 * (ai + an), pref = am * am * am * host::hubble_E(c, am);
        L.f1h = static_cast<float>(pref * host::growth_dD1(c, am));
        L.f2h = static_cast<float>(pref * host::growth_dD2(c, am));
      }
      L.tab = static_cast<const float*>(jp.data(tb.data(), tb.size() * sizeof(float)));
      L.reps = reps_dev;
      L.nrep = nact;
      L.out = reinterpret_cast<kern::LcRecord*>(lc->records);
      L.count = counter;
      L.capacity = lc->capacity;
    }
    jp.upload(s);
    run_cola(jp, f, tab, n_a, cosmo->omega_m, cola, flags, s, &lcs);
    unsigned long long cnt = 0;
    check(hipMemcpyAsync(&cnt, counter, sizeof(cnt), hipMemcpyDeviceToHost, s), "hipMemcpyAsync(count)");
    lpc_status st = finish(flags, s);
    *n_records = static_cast<int64_t>(cnt);
    if (st != LPC_OK) return st;
    if (static_cast<long long>(cnt) > lc->capacity)
      return fail(LPC_ERR_CAPACITY, "%llu lightcone records, capacity %lld: the records past the capacity were dropped",
                  cnt, static_cast<long long>(lc->capacity));
    return LPC_OK;
  });
}

// ---------------------------------------------------------------------------------------------------------------
// Batched form: workspace = flags, job region, then per box its int64/force mesh and three half spectra, then the
// sort space of all boxes (two tile-sorted copies of every box's particles, keys, ranks, tile counts and starts).
static bool batch_layout(const lpc_batch_entry* e, int32_t n_real, std::vector<size_t>* offs, size_t* total,
                         SortSpace* ss, void* ws) {
  if (!e || n_real < 1) return false;
  size_t off = round_up(sizeof(int) * kern::kNumFlags) + round_up(kJobRegion);
  if (offs) offs->clear();
  std::vector<int64_t> np;
  std::vector<int> nms;
  for (int i = 0; i < n_real; ++i) {
    const int nm = e[i].geom.n_mesh;
    if (!fft_size_ok(nm)) return false;
    const int64_t n = e[i].particles.n;
    if (n < 1 || n > (int64_t(1) << 31) - 1) return false;
    const size_t M = static_cast<size_t>(nm) * nm * nm;
    const size_t cbytes = round_up(static_cast<size_t>(nm) * nm * kern::mesh_pitch(nm) * sizeof(float2));
    if (offs) offs->push_back(off);
    off += round_up(M * 12) + 3 * cbytes;
    np.push_back(n);
    nms.push_back(nm);
  }
  int64_t ptot = 0;
  for (int64_t n : np) ptot += n;
  if (ptot > (int64_t(1) << 31) - 1) return false;
  off = layout_sort(static_cast<char*>(ws), off, np, nms, true, ss);
  *total = off;
  return true;
}

size_t lpc_workspace_bytes_batched(const lpc_batch_entry* entries, int32_t n_real) {
  size_t total = 0;
  return batch_layout(entries, n_real, nullptr, &total, nullptr, nullptr) ? total : 0;
}

lpc_status lpc_graph_enable(int32_t on) {
  g_graph_on = (on != 0);
  return LPC_OK;
}

lpc_status lpc_cola_step_batched(const lpc_batch_entry* entries, int32_t n_real, const lpc_cosmology* cosmo,
                                 const lpc_stepping* step, const double* a_list, int32_t n_a, void* ws,
                                 size_t ws_bytes, void* stream) {
  if (!entries || n_real < 1 || n_real > 4096) return fail(LPC_ERR_INVALID_ARG, "need 1..4096 batch entries");
  if (lpc_status st = check_cosmo(cosmo)) return st;
  if (lpc_status st = check_stepping(step)) return st;
  for (int i = 0; i < n_real; ++i) {
    if (lpc_status st = check_geom_mesh(&entries[i].geom)) return fail(st, "entry %d: %s", i, g_error.c_str());
    if (lpc_status st = check_particles(&entries[i].particles, step->cola != 0))
      return fail(st, "entry %d: %s", i, g_error.c_str());
    if (entries[i].particles.n == 0) return fail(LPC_ERR_INVALID_ARG, "entry %d has no particles", i);
  }
  std::vector<double> tab(static_cast<size_t>(n_a > 0 ? n_a : 0) * host::kCoefColumns);
  if (lpc_status st = lpc_cola_coefficients(cosmo, step, a_list, n_a, tab.data())) return st;
  std::vector<size_t> offs;
  size_t need = 0;
  SortSpace ss;
  if (!batch_layout(entries, n_real, &offs, &need, &ss, ws))
    return fail(LPC_ERR_INVALID_ARG, "batch has more than 2^31 - 1 particles in all");
  if (lpc_status st = check_ws(ws, ws_bytes, need)) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  return guarded([&]() {
    int* flags = reinterpret_cast<int*>(ws);
    stage("clear flags", s, [&] { return kern::fill_i32(flags, kern::kNumFlags, 0, s); });
    JobPack jp(at(ws, round_up(sizeof(int) * kern::kNumFlags)));  // the job region follows the flags
    std::vector<ForceBox> boxes;
    for (int i = 0; i < n_real; ++i) {
      const lpc_batch_entry& e = entries[i];
      const int nm = e.geom.n_mesh;
      const size_t M = static_cast<size_t>(nm) * nm * nm;
      const size_t cbytes = round_up(static_cast<size_t>(nm) * nm * kern::mesh_pitch(nm) * sizeof(float2));
      char* base = at(ws, offs[i]);
      ForceBox b{};
      b.nm = nm;
      b.box = e.geom.box;
      b.n = e.particles.n;
      b.pos = e.particles.pos;
      b.vel = e.particles.vel;
      b.psi1 = e.particles.psi1;
      b.psi2 = e.particles.psi2;
      b.dens = reinterpret_cast<uint64_t*>(base);
      b.force = reinterpret_cast<float*>(base);
      b.A = reinterpret_cast<float2*>(base + round_up(M * 12));
      b.B = reinterpret_cast<float2*>(base + round_up(M * 12) + cbytes);
      b.C = reinterpret_cast<float2*>(base + round_up(M * 12) + 2 * cbytes);
      boxes.push_back(b);
    }
    const ForceProgram f = add_force(jp, boxes, ss, step->deconv_power, true);
    jp.upload(s);
    const bool cola = step->cola != 0;
    if (!g_graph_on || g_prof.on) {
      run_cola(jp, f, tab, n_a, cosmo->omega_m, cola, flags, s);
      return finish(flags, s);
    }
    // Graph of the whole run, keyed by every argument that shapes the launches; replayed while they repeat.
    std::vector<char> key;
    auto put = [&key](const void* p, size_t n) {
      const char* c = static_cast<const char*>(p);
      key.insert(key.end(), c, c + n);
    };
    put(entries, sizeof(lpc_batch_entry) * n_real);
    put(cosmo, sizeof(*cosmo));
    put(step, sizeof(*step));
    put(a_list, sizeof(double) * n_a);
    put(&ws, sizeof(ws));
    const uint64_t tgen = tiling_generation();
    put(&tgen, sizeof(tgen));
    if (g_graph.exec == nullptr || g_graph.key != key) {
      if (g_graph.exec) {
        check(hipGraphExecDestroy(g_graph.exec), "hipGraphExecDestroy");
        g_graph.exec = nullptr;
      }
      kern::init_kernels();
      hipStream_t cap = capture_stream();
      hipGraph_t graph;
      check(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
      try {
        run_cola(jp, f, tab, n_a, cosmo->omega_m, cola, flags, cap);
      } catch (...) {
        hipGraph_t dropped = nullptr;  // end the capture so the stream is usable again; the error is the one thrown
        if (hipStreamEndCapture(cap, &dropped) == hipSuccess && dropped) (void)hipGraphDestroy(dropped);
        throw;
      }
      check(hipStreamEndCapture(cap, &graph), "hipStreamEndCapture");
      hipGraphExec_t exec;
      const hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      check(e, "hipGraphInstantiate");
      g_graph.exec = exec;
      g_graph.key = key;
    }
    check(hipGraphLaunch(g_graph.exec, s), "hipGraphLaunch");
    return finish(flags, s);
  });
}

lpc_status lpc_png_preset(int32_t kind, double f_nl, lpc_png* out) {
  if (!out) return fail(LPC_ERR_INVALID_ARG, "out is NULL");
  if (!std::isfinite(f_nl)) return fail(LPC_ERR_INVALID_ARG, "f_nl not finite");
  lpc_png p{};
  p.f_nl = f_nl;
  // (c, a, b, g) of NL = sum c D^g[(D^a phi)(D^b phi)]: the kernels whose bispectra are the published templates
  switch (kind) {
    case LPC_PNG_LOCAL:
      p.n_terms = 1;
      p.terms[0] = lpc_png_term{1.0, 0.0, 0.0, 0.0};
      break;
    case LPC_PNG_EQUILATERAL:
      p.n_terms = 3;
      p.terms[0] = lpc_png_term{-3.0, 0.0, 0.0, 0.0};
      p.terms[1] = lpc_png_term{6.0, 1.0, 0.0, -1.0};
      p.terms[2] = lpc_png_term{-2.0, 1.0, 1.0, -2.0};
      break;
    case LPC_PNG_ORTHOGONAL:
      p.n_terms = 3;
      p.terms[0] = lpc_png_term{-9.0, 0.0, 0.0, 0.0};
      p.terms[1] = lpc_png_term{18.0, 1.0, 0.0, -1.0};
      p.terms[2] = lpc_png_term{-8.0, 1.0, 1.0, -2.0};
      break;
    default:
      return fail(LPC_ERR_INVALID_ARG, "unknown non-Gaussianity kind %d", kind);
  }
  *out = p;
  return LPC_OK;
}

}  // extern "C"

namespace {

lpc_status check_png(const lpc_png* png) {
  if (!std::isfinite(png->f_nl)) return fail(LPC_ERR_INVALID_ARG, "f_nl not finite");
  if (png->n_terms < 1 || png->n_terms > kern::kPngMaxTerms)
    return fail(LPC_ERR_INVALID_ARG, "n_terms must be in [1, %d]", kern::kPngMaxTerms);
  if (png->reserved != 0) return fail(LPC_ERR_INVALID_ARG, "png.reserved must be 0");
  for (int t = 0; t < png->n_terms; ++t) {
    const lpc_png_term& q = png->terms[t];
    if (!std::isfinite(q.c) || !(std::fabs(q.a) <= 4.0) || !(std::fabs(q.b) <= 4.0) || !(std::fabs(q.g) <= 4.0))
      return fail(LPC_ERR_INVALID_ARG, "term %d: c must be finite and a, b, g within [-4, 4]", t);
  }
  return LPC_OK;
}

// 2LPT initial conditions; png (nullable) adds primordial non-Gaussianity to the linear field.
lpc_status init_ic_impl(const lpc_geometry* geom, const lpc_cosmology* cosmo, uint64_t seed, double a_init,
                        const lpc_png* png, const lpc_particles* out, void* ws, size_t ws_bytes, void* stream) {
  if (!geom) return fail(LPC_ERR_INVALID_ARG, "geometry is NULL");
  if (!(geom->box > 0.0) || !std::isfinite(geom->box)) return fail(LPC_ERR_INVALID_ARG, "box must be positive");
  if (lpc_status st = check_mesh(geom->n_side, "n_side")) return st;
  if (lpc_status st = check_cosmo(cosmo)) return st;
  if (!(a_init > 0.0) || !std::isfinite(a_init)) return fail(LPC_ERR_INVALID_ARG, "a_init must be positive");
  if (lpc_status st = check_particles(out, true)) return st;
  if (!out->id) return fail(LPC_ERR_INVALID_ARG, "id is NULL");
  if (png)
    if (lpc_status st = check_png(png)) return st;
  const int N = geom->n_side;
  const int64_t n = static_cast<int64_t>(N) * N * N;
  if (out->n != n) return fail(LPC_ERR_INVALID_ARG, "particles.n = %lld but n_side^3 = %lld",
                               static_cast<long long>(out->n), static_cast<long long>(n));
  // the distinct D exponents of the non-Gaussian terms (each needs one real field; five slots are free)
  std::vector<double> alphas, gammas;
  if (png) {
    for (int t = 0; t < png->n_terms; ++t) {
      for (double v : {png->terms[t].a, png->terms[t].b})
        if (std::find(alphas.begin(), alphas.end(), v) == alphas.end()) alphas.push_back(v);
      if (std::find(gammas.begin(), gammas.end(), png->terms[t].g) == gammas.end()) gammas.push_back(png->terms[t].g);
    }
    if (alphas.size() > 5) return fail(LPC_ERR_INVALID_ARG, "more than 5 distinct inner exponents a, b");
  }
  const Plan p = make_ws_plan(N, LPC_OP_INIT_IC, 0);
  if (lpc_status st = check_ws(ws, ws_bytes, p.total)) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  return guarded([&]() {
    const host::Cosmo c = to_host(cosmo);
    const double A = host::pk_amplitude(c);
    int* flags = reinterpret_cast<int*>(ws);
    stage("clear flags", s, [&] { return kern::fill_i32(flags, kern::kNumFlags, 0, s); });
    const int pitch = kern::mesh_pitch(N);
    float2* dhat = reinterpret_cast<float2*>(at(ws, p.A));
    float2* spec = reinterpret_cast<float2*>(at(ws, p.B));
    float2* nlhat = reinterpret_cast<float2*>(at(ws, p.C));
    float* r0 = out->psi2;
    float* r1 = out->psi2 + n;
    float* r2 = out->psi2 + 2 * n;
    const float inv_n3 = static_cast<float>(1.0 / static_cast<double>(n));
    // the transforms of the whole construction, in order: r2c(noise), 12 derived fields, r2c(source), and the 2LPT
    // displacement fields; kinds 0..2 Psi1, 3..8 phi1_ij, 9..11 Psi2
    float* dst[12] = {out->psi1, out->psi1 + n, out->psi1 + 2 * n, r0, r1, r2, r1, r1, r1, r0, r1, r2};
    JobPack jp(at(ws, p.jobs));
    const R2CSections noise = add_r2c(jp, r0, false, 0.0, N, dhat);
    C2RSections der[12];
    for (int k = 0; k < 12; ++k) der[k] = add_c2r(jp, spec, N, dst[k], inv_n3);
    const R2CSections source = add_r2c(jp, r0, false, 0.0, N, dhat);
    // non-Gaussian stage: real fields D^a phi in the five slots psi1[0..2], psi2[1..2]; products in psi2[0]
    float* slot[5] = {out->psi1, out->psi1 + n, out->psi1 + 2 * n, r1, r2};
    std::vector<C2RSections> to_real;
    std::vector<R2CSections> prod_r2c;
    for (size_t v = 0; v < alphas.size(); ++v) to_real.push_back(add_c2r(jp, spec, N, slot[v], inv_n3));
    for (size_t v = 0; v < gammas.size(); ++v) prod_r2c.push_back(add_r2c(jp, r0, false, 0.0, N, spec));
    jp.upload(s);
    auto derived = [&](int kind) {
      stage("spectral factor", s, [&] { return kern::ic_spectral_factor(dhat, spec, N, pitch, geom->box, kind, s); });
      run_c2r(jp, der[kind], s);
    };
    stage("noise", s, [&] { return kern::ic_noise(seed, N, r0, s); });
    run_r2c(jp, noise, false, flags, s);
    if (!png) {
      stage("scale spectrum", s, [&] { return kern::ic_scale_spectrum(dhat, N, pitch, geom->box, A, c.omega_m, c.h, c.n_s, s); });
    } else {
      // Phi = phi + fNL sum_j c_j D^g[(D^a phi)(D^b phi)], D^s = k^(s (4 - ns) / 3); delta_L = alpha0 k^2 T Phi
      const double g0 = host::growth_suppression(c);
      const double alpha0 = (2.0 / 3.0) * host::kCOverH0 * host::kCOverH0 * g0 / c.omega_m;
      const double a_phi = A / (alpha0 * alpha0);
      const double tilt = (4.0 - c.n_s) / 3.0;
      stage("png potential", s, [&] { return kern::png_potential(dhat, N, pitch, geom->box, a_phi, c.n_s, s); });
      for (size_t v = 0; v < alphas.size(); ++v) {
        stage("png power", s, [&] {
          return kern::png_power(dhat, spec, N, pitch, geom->box, alphas[v] * tilt, 1.0, false, s);
        });
        run_c2r(jp, to_real[v], s);
      }
      auto field = [&](double e) {
        return slot[std::find(alphas.begin(), alphas.end(), e) - alphas.begin()];
      };
      for (size_t gi = 0; gi < gammas.size(); ++gi) {
        kern::PngProducts pp{};
        pp.out = r0;
        for (int t = 0; t < png->n_terms; ++t) {
          if (png->terms[t].g != gammas[gi]) continue;
          pp.fa[pp.n] = field(png->terms[t].a);
          pp.fb[pp.n] = field(png->terms[t].b);
          pp.c[pp.n] = static_cast<float>(png->terms[t].c);
          ++pp.n;
        }
        stage("png products", s, [&] { return kern::png_products(pp, n, s); });
        run_r2c(jp, prod_r2c[gi], false, flags, s);
        stage("png power", s, [&] {
          return kern::png_power(spec, nlhat, N, pitch, geom->box, gammas[gi] * tilt, 1.0, gi > 0, s);
        });
      }
      stage("png to delta", s, [&] {
        return kern::png_to_delta(dhat, nlhat, N, pitch, geom->box, png->f_nl, alpha0, c.omega_m, c.h, s);
      });
    }
    for (int k = 0; k < 3; ++k) derived(k);  // Psi1
    for (int k = 3; k < 6; ++k) derived(k);  // phi_xx, phi_yy, phi_zz
    stage("source", s, [&] { return kern::ic_source_init(r0, r1, r2, n, s); });
    for (int k = 6; k < 9; ++k) {            // phi_xy, phi_xz, phi_yz
      derived(k);
      stage("source", s, [&] { return kern::ic_sub_square(r0, r1, n, s); });
    }
    run_r2c(jp, source, false, flags, s);    // source spectrum replaces delta_hat
    // Psi2 = i k phi2_hat; kinds 9..11 read the source spectrum in dhat
    for (int j = 0; j < 3; ++j) {
      stage("spectral factor", s, [&] { return kern::ic_spectral_factor(dhat, spec, N, pitch, geom->box, 9 + j, s); });
      run_c2r(jp, der[9 + j], s);
    }
    const double d1 = host::growth_D1(c, a_init), d2 = host::growth_D2(c, a_init);
    const double E = host::hubble_E(c, a_init), a3 = a_init * a_init * a_init;
    const double f1 = a3 * E * host::growth_dD1(c, a_init), f2 = a3 * E * host::growth_dD2(c, a_init);
    stage("assemble", s, [&] {
      return kern::ic_assemble(out->pos, out->vel, out->id, out->psi1, out->psi2, N, geom->box, static_cast<float>(d1),
                               static_cast<float>(d2), static_cast<float>(f1), static_cast<float>(f2), s);
    });
    return finish(flags, s);
  });
}

}  // namespace

namespace {

// Tile sort, fixed-point deposit (FP32 contrast in the density region) and forward r2c into A: the density
// spectrum of a statistic's particles, on workspace plan p of operation op.
struct DensitySpectrum {
  SortSpace ss;
  Section sort, dep;
  R2CSections r;
};

DensitySpectrum add_density_spectrum(JobPack& jp, void* ws, const Plan& p, const lpc_geometry* geom, const float* pos,
                                     int64_t n, int op, float2* A) {
  DensitySpectrum d;
  const int nm = geom->n_mesh;
  const int64_t M = static_cast<int64_t>(nm) * nm * nm;
  d.ss = sort_space(ws, p, nm, op, n);
  const kern::TileGrid nt = d.ss.nt[0];
  kern::SortJob sj{};
  sj.pos = pos;
  sj.dpos = d.ss.copy[0][0].pos;
  sj.dorig = d.ss.copy[0][0].orig;
  sj.n = n;
  sj.ntx = nt.x;
  sj.nty = nt.y;
  sj.ntz = nt.z;
  sj.nm = nm;
  sj.scale = (static_cast<double>(nm) * 65536.0) / geom->box;
  d.sort = jp.add1(sj, static_cast<int>((n + kern::kNT - 1) / kern::kNT));
  kern::DepJob dj{};
  dj.pos = sj.dpos;
  dj.n = n;
  dj.ntx = nt.x;
  dj.nty = nt.y;
  dj.ntz = nt.z;
  dj.inv_yz = kern::div_inverse(nt.y * nt.z);
  dj.inv_z = kern::div_inverse(nt.z);
  dj.nm = nm;
  dj.scale = sj.scale;
  dj.delta = reinterpret_cast<float*>(at(ws, p.dens));  // the FP32 contrast, in the density region
  dj.mscale = (static_cast<double>(M) / static_cast<double>(n)) * 0x1.0p-48;
  d.dep = jp.add1(dj, nt.count());
  d.r = add_r2c(jp, dj.delta, false, 0.0, nm, A);
  return d;
}

void run_density_spectrum(const JobPack& jp, const DensitySpectrum& d, int* flags, hipStream_t s) {
  run_sort(jp, d.ss, d.sort, flags, s);
  stage("deposit", s, [&] {
    return kern::launch_deposit_tiles(jp.jobs<kern::DepJob>(d.dep), jp.table(d.dep), d.ss.start, flags, s);
  });
  run_r2c(jp, d.r, false, flags, s);
}

}  // namespace

extern "C" {

lpc_status lpc_init_ic(const lpc_geometry* geom, const lpc_cosmology* cosmo, uint64_t seed, double a_init,
                       const lpc_particles* out, void* ws, size_t ws_bytes, void* stream) {
  return init_ic_impl(geom, cosmo, seed, a_init, nullptr, out, ws, ws_bytes, stream);
}

lpc_status lpc_init_ic_png(const lpc_geometry* geom, const lpc_cosmology* cosmo, uint64_t seed, double a_init,
                           const lpc_png* png, const lpc_particles* out, void* ws, size_t ws_bytes, void* stream) {
  if (!png) return fail(LPC_ERR_INVALID_ARG, "png is NULL");
  return init_ic_impl(geom, cosmo, seed, a_init, png, out, ws, ws_bytes, stream);
}

lpc_status lpc_power_spectrum(const lpc_geometry* geom, const float* pos, int64_t n, double k_max, int32_t n_bins,
                              double* k_mean, double* pk, int64_t* n_modes, void* ws, size_t ws_bytes, void* stream) {
  if (lpc_status st = check_geom_mesh(geom)) return st;
  if (n <= 0 || n > (int64_t(1) << 31) - 1) return fail(LPC_ERR_INVALID_ARG, "n must be in [1, 2^31 - 1]");
  if (!pos || !k_mean || !pk || !n_modes) return fail(LPC_ERR_INVALID_ARG, "NULL array");
  if (n_bins < 1 || n_bins > 2048) return fail(LPC_ERR_INVALID_ARG, "n_bins must be in [1, 2048]");
  if (!(k_max > 0.0) || !std::isfinite(k_max)) return fail(LPC_ERR_INVALID_ARG, "k_max must be positive");
  const Plan p = make_ws_plan(geom->n_mesh, LPC_OP_POWER_SPECTRUM, n);
  if (lpc_status st = check_ws(ws, ws_bytes, p.total)) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  return guarded([&]() {
    const int nm = geom->n_mesh, pitch = kern::mesh_pitch(nm);
    const int64_t M = static_cast<int64_t>(nm) * nm * nm;
    int* flags = reinterpret_cast<int*>(ws);
    float2* A = reinterpret_cast<float2*>(at(ws, p.A));
    double* sums = reinterpret_cast<double*>(at(ws, p.bins));
    unsigned long long* counts = reinterpret_cast<unsigned long long*>(sums + 2 * n_bins);
    JobPack jp(at(ws, p.jobs));
    const DensitySpectrum ds = add_density_spectrum(jp, ws, p, geom, pos, n, LPC_OP_POWER_SPECTRUM, A);
    jp.upload(s);
    stage("clear flags", s, [&] { return kern::fill_i32(flags, kern::kNumFlags, 0, s); });
    stage("clear bins", s, [&] {
      return kern::fill_i32(reinterpret_cast<int*>(sums), static_cast<size_t>(6) * n_bins, 0, s);
    });
    run_density_spectrum(jp, ds, flags, s);
    const double V = geom->box * geom->box * geom->box;
    const double pscale = V / (static_cast<double>(M) * static_cast<double>(M));
    stage("pk bin", s, [&] { return kern::pk_bin(A, nm, pitch, geom->box, k_max, n_bins, pscale, sums, counts, s); });
    std::vector<double> hs(static_cast<size_t>(3) * n_bins);
    check(hipMemcpyAsync(hs.data(), sums, hs.size() * sizeof(double), hipMemcpyDeviceToHost, s), "copy bins");
    lpc_status st = finish(flags, s);
    if (st != LPC_OK) return st;
    const unsigned long long* hc = reinterpret_cast<const unsigned long long*>(hs.data() + 2 * n_bins);
    for (int b = 0; b < n_bins; ++b) {
      n_modes[b] = static_cast<int64_t>(hc[b]);
      if (hc[b] == 0) {
        k_mean[b] = pk[b] = std::nan("");
      } else {
        k_mean[b] = hs[2 * b] / static_cast<double>(hc[b]);
        pk[b] = hs[2 * b + 1] / static_cast<double>(hc[b]);
      }
    }
    return LPC_OK;
  });
}

lpc_status lpc_bispectrum(const lpc_geometry* geom, const float* pos, int64_t n, const double* k123, int32_t m,
                          double dk, double* B, double* Q, double* P, void* ws, size_t ws_bytes, void* stream) {
  if (lpc_status st = check_geom_mesh(geom)) return st;
  if (n <= 0 || n > (int64_t(1) << 31) - 1) return fail(LPC_ERR_INVALID_ARG, "n must be in [1, 2^31 - 1]");
  if (!pos || !k123 || !B || !Q) return fail(LPC_ERR_INVALID_ARG, "NULL array");
  if (m < 1 || m > kMaxTriangles) return fail(LPC_ERR_INVALID_ARG, "m must be in [1, %d]", kMaxTriangles);
  if (!(dk > 0.0) || !std::isfinite(dk)) return fail(LPC_ERR_INVALID_ARG, "dk must be positive");
  for (int t = 0; t < 3 * m; ++t)
    if (!(k123[t] > 0.0) || !std::isfinite(k123[t])) return fail(LPC_ERR_INVALID_ARG, "shell centres must be positive");
  const Plan p = make_ws_plan(geom->n_mesh, LPC_OP_BISPECTRUM, n);
  if (lpc_status st = check_ws(ws, ws_bytes, p.total)) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  return guarded([&]() {
    const int nm = geom->n_mesh, pitch = kern::mesh_pitch(nm);
    const int64_t M = static_cast<int64_t>(nm) * nm * nm;
    const double box = geom->box;
    int* flags = reinterpret_cast<int*>(ws);
    float2* A = reinterpret_cast<float2*>(at(ws, p.A));
    float2* H = reinterpret_cast<float2*>(at(ws, p.B));
    float* F[3];
    for (int i = 0; i < 3; ++i) F[i] = reinterpret_cast<float*>(at(ws, p.fields)) + i * M;
    double* parts = reinterpret_cast<double*>(at(ws, p.bins));
    const int nb = kern::sum_blocks();
    JobPack jp(at(ws, p.jobs));
    const DensitySpectrum ds = add_density_spectrum(jp, ws, p, geom, pos, n, LPC_OP_BISPECTRUM, A);
    // the unnormalised inverse transform of H into each of the three real meshes (H is consumed each time)
    const C2RSections inv[3] = {add_c2r(jp, H, nm, F[0], 1.f), add_c2r(jp, H, nm, F[1], 1.f),
                                add_c2r(jp, H, nm, F[2], 1.f)};
    jp.upload(s);
    stage("clear flags", s, [&] { return kern::fill_i32(flags, kern::kNumFlags, 0, s); });
    run_density_spectrum(jp, ds, flags, s);
    for (int t = 0; t < m; ++t) {
      double* pt = parts + static_cast<size_t>(t) * kPartsPerTriangle * nb;
      for (int ind = 0; ind < 2; ++ind) {  // shell-filtered fields, then the shell indicators
        for (int i = 0; i < 3; ++i) {
          const double kc = k123[3 * t + i];
          stage("shell fill", s, [&] {
            return kern::shell_fill(A, H, nm, pitch, box, kc - 0.5 * dk, kc + 0.5 * dk, ind == 1, s);
          });
          run_c2r(jp, inv[i], s);
        }
        stage("triple sum", s, [&] { return kern::triple_sum(F[0], F[1], F[2], M, pt + ind * nb, s); });
      }
      for (int i = 0; i < 3; ++i) {
        const double kc = k123[3 * t + i];
        stage("shell power", s, [&] {
          return kern::shell_power(A, nm, pitch, box, kc - 0.5 * dk, kc + 0.5 * dk, pt + (2 + 2 * i) * nb,
                                   pt + (3 + 2 * i) * nb, s);
        });
      }
    }
    std::vector<double> hp(static_cast<size_t>(m) * kPartsPerTriangle * nb);
    check(hipMemcpyAsync(hp.data(), parts, hp.size() * sizeof(double), hipMemcpyDeviceToHost, s), "copy sums");
    lpc_status st = finish(flags, s);
    if (st != LPC_OK) return st;
    const double V = box * box * box, Md = static_cast<double>(M);
    for (int t = 0; t < m; ++t) {
      double sum[kPartsPerTriangle] = {};
      for (int q = 0; q < kPartsPerTriangle; ++q)
        for (int b = 0; b < nb; ++b) sum[q] += hp[(static_cast<size_t>(t) * kPartsPerTriangle + q) * nb + b];
      double pw[3];
      for (int i = 0; i < 3; ++i) pw[i] = (sum[3 + 2 * i] > 0.0) ? V / (Md * Md) * sum[2 + 2 * i] / sum[3 + 2 * i] : std::nan("");
      // sum_x I1 I2 I3 is Nm^3 times the number of closed triangles (exact up to FP32 rounding of the fields)
      B[t] = (sum[1] >= 0.5 * Md) ? V * V / (Md * Md * Md) * sum[0] / sum[1] : std::nan("");
      Q[t] = B[t] / (pw[0] * pw[1] + pw[1] * pw[2] + pw[2] * pw[0]);
      if (P)
        for (int i = 0; i < 3; ++i) P[3 * t + i] = pw[i];
    }
    return LPC_OK;
  });
}

lpc_status lpc_fft_r2c(int32_t n, const float* in, float* out_complex, void* ws, size_t ws_bytes, void* stream) {
  if (lpc_status st = check_mesh(n, "n")) return st;
  if (!in || !out_complex) return fail(LPC_ERR_INVALID_ARG, "NULL array");
  const Plan p = make_ws_plan(n, LPC_OP_FFT, 0);
  if (lpc_status st = check_ws(ws, ws_bytes, p.total)) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  return guarded([&]() {
    int* flags = reinterpret_cast<int*>(ws);
    stage("clear flags", s, [&] { return kern::fill_i32(flags, kern::kNumFlags, 0, s); });
    JobPack jp(at(ws, p.jobs));
    const R2CSections r = add_r2c(jp, in, false, 0.0, n, reinterpret_cast<float2*>(out_complex));
    jp.upload(s);
    run_r2c(jp, r, false, flags, s);
    return finish(flags, s);
  });
}

lpc_status lpc_fft_c2r(int32_t n, float* in_complex, float* out, void* ws, size_t ws_bytes, void* stream) {
  if (lpc_status st = check_mesh(n, "n")) return st;
  if (!in_complex || !out) return fail(LPC_ERR_INVALID_ARG, "NULL array");
  const Plan p = make_ws_plan(n, LPC_OP_FFT, 0);
  if (lpc_status st = check_ws(ws, ws_bytes, p.total)) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  return guarded([&]() {
    int* flags = reinterpret_cast<int*>(ws);
    stage("clear flags", s, [&] { return kern::fill_i32(flags, kern::kNumFlags, 0, s); });
    JobPack jp(at(ws, p.jobs));
    const C2RSections c = add_c2r(jp, reinterpret_cast<float2*>(in_complex), n, out, 1.0f);
    jp.upload(s);
    run_c2r(jp, c, s);
    return finish(flags, s);
  });
}

}  // extern "C"
