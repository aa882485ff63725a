// C ABI of liblpc (declared in include/lpc.h): argument checks, the workspace plan, the FP64 coefficient table and
// the sequence of kernel launches for each entry point. No C++ exception crosses this boundary.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <exception>
#include <string>
#include <vector>

#include "../../include/lpc.h"
#include "lpc_host.h"
#include "lpc_kernels.h"

namespace {

using lpc::kern::Plan1D;
namespace kern = lpc::kern;
namespace host = lpc::host;

thread_local std::string g_error;

lpc_status fail(lpc_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_error = buf;
  return s;
}

struct HipError {
  hipError_t e;
  const char* what;
};

void check(hipError_t e, const char* what) {
  if (e != hipSuccess) throw HipError{e, what};
}

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

bool fft_size_ok(int n) {
  if (n < 8 || n > 1024 || (n % 2) != 0) return false;
  Plan1D p;
  return kern::make_plan(n, &p) && kern::make_plan(n / 2, &p);
}

// Workspace plan of one operation on an n^3 mesh: flags first, then 256-byte aligned regions.
struct Plan {
  size_t flags = 0, dens = 0, A = 0, B = 0, C = 0, bins = 0, total = 0;
  size_t complex_elems = 0;  // float2 per complex mesh
};

Plan make_ws_plan(int n, int op, int n_bins = 0) {
  Plan p;
  const size_t M = static_cast<size_t>(n) * n * n;
  p.complex_elems = static_cast<size_t>(n) * n * kern::mesh_pitch(n);
  const size_t cbytes = round_up(p.complex_elems * sizeof(float2));
  size_t off = round_up(sizeof(int) * kern::kNumFlags);
  auto take = [&off](size_t bytes) {
    size_t at = off;
    off += round_up(bytes);
    return at;
  };
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
      break;
    case LPC_OP_POWER_SPECTRUM:
      p.dens = take(M * 8);
      p.A = take(cbytes);
      p.bins = take(static_cast<size_t>(n_bins > 0 ? n_bins : 2048) * 3 * sizeof(double));
      break;
    case LPC_OP_FFT:
      break;
    default:
      return Plan{};
  }
  p.total = off;
  return p;
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

template <class F>
lpc_status guarded(F body) {
  try {
    return body();
  } catch (const HipError& e) {
    return fail(LPC_ERR_HIP, "%s failed: %s", e.what, hipGetErrorString(e.e));
  } catch (const std::exception& e) {
    return fail(LPC_ERR_HIP, "internal error: %s", e.what());
  } catch (...) {
    return fail(LPC_ERR_HIP, "unknown internal error");
  }
}

char* at(void* ws, size_t off) { return static_cast<char*>(ws) + off; }

// Forward r2c of an FP32 real mesh, then y and x passes (in place on `out`).
void r2c_real(const float* in, int n, float2* out, hipStream_t s) {
  const int pitch = kern::mesh_pitch(n), nh = n / 2 + 1;
  stage("fft z r2c", s, [&] { return kern::fft_z_r2c_real(in, n, out, pitch, s); });
  stage("fft y", s, [&] { return kern::fft_axis(out, n, pitch, static_cast<int64_t>(n) * pitch, n, nh, 1, 0, false, s); });
  stage("fft x", s, [&] { return kern::fft_axis(out, n, static_cast<int64_t>(n) * pitch, pitch, n, nh, 1, 0, false, s); });
}

// Inverse x and y passes in place on `spec`, then c2r into `out` times `scale`.
void c2r_real(float2* spec, int n, float* out, float scale, hipStream_t s) {
  const int pitch = kern::mesh_pitch(n), nh = n / 2 + 1;
  stage("fft x inv", s, [&] { return kern::fft_axis(spec, n, static_cast<int64_t>(n) * pitch, pitch, n, nh, 1, 0, true, s); });
  stage("fft y inv", s, [&] { return kern::fft_axis(spec, n, pitch, static_cast<int64_t>(n) * pitch, n, nh, 1, 0, true, s); });
  stage("fft z c2r", s, [&] { return kern::fft_z_c2r_real(spec, n, pitch, out, scale, s); });
}

// The mesh part of the PM force: deposit -> delta -> FFT -> Poisson/gradient -> 3 inverse FFTs -> AoS force mesh.
// Returns the force mesh (float[nm^3][3]) in the workspace.
float* force_mesh(const float* pos, int64_t n, int nm, double box, int deconv, void* ws, const Plan& p,
                  uint64_t* dens_override, int* flags, hipStream_t s) {
  const size_t M = static_cast<size_t>(nm) * nm * nm;
  const int pitch = kern::mesh_pitch(nm), nh = nm / 2 + 1;
  uint64_t* dens = dens_override ? dens_override : reinterpret_cast<uint64_t*>(at(ws, p.dens));
  float2* A = reinterpret_cast<float2*>(at(ws, p.A));
  float2* B = reinterpret_cast<float2*>(at(ws, p.B));
  float2* C = reinterpret_cast<float2*>(at(ws, p.C));
  float* force = reinterpret_cast<float*>(at(ws, p.dens));
  const double scale = (static_cast<double>(nm) * 65536.0) / box;
  const double mscale = (static_cast<double>(M) / static_cast<double>(n)) * 0x1.0p-48;
  stage("fill density", s, [&] { return kern::fill_u64(dens, M, s); });
  stage("deposit", s, [&] { return kern::deposit(pos, n, nm, scale, dens, flags, s); });
  stage("fft z r2c", s, [&] { return kern::fft_z_r2c_fixed(dens, nm, mscale, A, pitch, flags, s); });
  stage("fft y", s, [&] { return kern::fft_axis(A, nm, pitch, static_cast<int64_t>(nm) * pitch, nm, nh, 1, 0, false, s); });
  stage("fft x + poisson", s, [&] { return kern::fft_x_poisson(A, B, C, nm, pitch, box, deconv, s); });
  const int64_t cstride = static_cast<int64_t>(B - A);
  if (C - B != B - A) throw HipError{hipErrorInvalidValue, "workspace layout"};
  stage("fft y inv", s, [&] { return kern::fft_axis(A, nm, pitch, static_cast<int64_t>(nm) * pitch, nm, nh, 3, cstride, true, s); });
  stage("fft z c2r", s, [&] { return kern::fft_z_c2r_aos3(A, B, C, nm, pitch, force, s); });
  return force;
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

}  // namespace

extern "C" {

size_t lpc_workspace_bytes(const lpc_geometry* geom, int32_t op) {
  if (!geom) return 0;
  const int n = (op == LPC_OP_INIT_IC) ? geom->n_side : geom->n_mesh;
  if (!fft_size_ok(n)) return 0;
  return make_ws_plan(n, op).total;
}

int32_t lpc_fft_pitch(int32_t n) { return (n >= 2) ? kern::mesh_pitch(n) : 0; }

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
  }
  return "unknown lpc_status";
}

const char* lpc_last_error(void) { return g_error.c_str(); }

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
  if (lpc_status st = check_geom_mesh(geom)) return st;
  if (!step) return fail(LPC_ERR_INVALID_ARG, "stepping is NULL");
  if (step->deconv_power < 0 || step->deconv_power > 2) return fail(LPC_ERR_INVALID_ARG, "deconv_power not in 0..2");
  if (n <= 0 || n > (int64_t(1) << 31) - 1) return fail(LPC_ERR_INVALID_ARG, "n must be in [1, 2^31 - 1]");
  if (!pos || !grad_out) return fail(LPC_ERR_INVALID_ARG, "pos/grad_out is NULL");
  const Plan p = make_ws_plan(geom->n_mesh, LPC_OP_PM_FORCE);
  if (lpc_status st = check_ws(ws, ws_bytes, p.total)) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  return guarded([&]() {
    int* flags = reinterpret_cast<int*>(ws);
    stage("clear flags", s, [&] { return kern::fill_i32(flags, kern::kNumFlags, 0, s); });
    const int nm = geom->n_mesh;
    float* F = force_mesh(pos, n, nm, geom->box, step->deconv_power, ws, p,
                          reinterpret_cast<uint64_t*>(density_fixed_out), flags, s);
    const double scale = (static_cast<double>(nm) * 65536.0) / geom->box;
    stage("gather", s, [&] { return kern::gather(pos, n, F, nm, scale, grad_out, flags, s); });
    return finish(flags, s);
  });
}

lpc_status lpc_cola_step(const lpc_geometry* geom, const lpc_cosmology* cosmo, const lpc_stepping* step,
                         const double* a_list, int32_t n_a, const lpc_particles* inout, void* ws, size_t ws_bytes,
                         void* stream) {
  if (lpc_status st = check_geom_mesh(geom)) return st;
  if (lpc_status st = check_cosmo(cosmo)) return st;
  if (!step) return fail(LPC_ERR_INVALID_ARG, "stepping is NULL");
  if (step->deconv_power < 0 || step->deconv_power > 2) return fail(LPC_ERR_INVALID_ARG, "deconv_power not in 0..2");
  if (step->reserved != 0) return fail(LPC_ERR_INVALID_ARG, "stepping.reserved must be 0");
  if (lpc_status st = check_particles(inout, step->cola != 0)) return st;
  if (inout->n == 0) return fail(LPC_ERR_INVALID_ARG, "no particles");
  std::vector<double> tab(static_cast<size_t>(n_a > 0 ? n_a : 0) * host::kCoefColumns);
  if (lpc_status st = lpc_cola_coefficients(cosmo, step, a_list, n_a, tab.data())) return st;
  const Plan p = make_ws_plan(geom->n_mesh, LPC_OP_COLA_STEP);
  if (lpc_status st = check_ws(ws, ws_bytes, p.total)) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  return guarded([&]() {
    int* flags = reinterpret_cast<int*>(ws);
    stage("clear flags", s, [&] { return kern::fill_i32(flags, kern::kNumFlags, 0, s); });
    const int nm = geom->n_mesh;
    const int64_t n = inout->n;
    const bool cola = step->cola != 0;
    const double om = cosmo->omega_m;
    const double scale = (static_cast<double>(nm) * 65536.0) / geom->box;
    auto row = [&tab](int i) { return tab.data() + static_cast<size_t>(i) * host::kCoefColumns; };
    if (cola)
      stage("frame velocity", s, [&] { return kern::frame_velocity(inout->vel, inout->psi1, inout->psi2, n, static_cast<float>(-row(0)[host::kF1]),
                                 static_cast<float>(-row(0)[host::kF2]), s); });
    for (int i = 0; i < n_a; ++i) {
      const double* r = row(i);
      float* F = force_mesh(inout->pos, n, nm, geom->box, step->deconv_power, ws, p, nullptr, flags, s);
      kern::KickDrift kd;
      kd.kick = static_cast<float>(r[host::kK] * (-1.5 * om));
      kd.d1 = static_cast<float>(r[host::kD1]);
      kd.d2m = static_cast<float>(r[host::kD2] - r[host::kD1] * r[host::kD1]);
      kd.drift = static_cast<float>(r[host::kQ]);
      kd.dd1 = static_cast<float>(r[host::kDD1]);
      kd.dd2 = static_cast<float>(r[host::kDD2]);
      kd.do_drift = (i + 1 < n_a) ? 1 : 0;
      kd.cola = cola ? 1 : 0;
      stage("gather kick drift", s, [&] { return kern::gather_kick_drift(inout->pos, inout->vel, inout->psi1, inout->psi2, n, F, nm, scale,
                                    static_cast<float>(geom->box), kd, flags, s); });
    }
    if (cola) {
      const double* r = row(n_a - 1);
      stage("frame velocity", s, [&] { return kern::frame_velocity(inout->vel, inout->psi1, inout->psi2, n, static_cast<float>(r[host::kF1]),
                                 static_cast<float>(r[host::kF2]), s); });
    }
    return finish(flags, s);
  });
}

lpc_status lpc_init_ic(const lpc_geometry* geom, const lpc_cosmology* cosmo, uint64_t seed, double a_init,
                       const lpc_particles* out, void* ws, size_t ws_bytes, void* stream) {
  if (!geom) return fail(LPC_ERR_INVALID_ARG, "geometry is NULL");
  if (!(geom->box > 0.0) || !std::isfinite(geom->box)) return fail(LPC_ERR_INVALID_ARG, "box must be positive");
  if (lpc_status st = check_mesh(geom->n_side, "n_side")) return st;
  if (lpc_status st = check_cosmo(cosmo)) return st;
  if (!(a_init > 0.0) || !std::isfinite(a_init)) return fail(LPC_ERR_INVALID_ARG, "a_init must be positive");
  if (lpc_status st = check_particles(out, true)) return st;
  if (!out->id) return fail(LPC_ERR_INVALID_ARG, "id is NULL");
  const int N = geom->n_side;
  const int64_t n = static_cast<int64_t>(N) * N * N;
  if (out->n != n) return fail(LPC_ERR_INVALID_ARG, "particles.n = %lld but n_side^3 = %lld",
                               static_cast<long long>(out->n), static_cast<long long>(n));
  const Plan p = make_ws_plan(N, LPC_OP_INIT_IC);
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
    float* r0 = out->psi2;
    float* r1 = out->psi2 + n;
    float* r2 = out->psi2 + 2 * n;
    const float inv_n3 = static_cast<float>(1.0 / static_cast<double>(n));
    stage("noise", s, [&] { return kern::ic_noise(seed, N, r0, s); });
    r2c_real(r0, N, dhat, s);
    stage("scale spectrum", s, [&] { return kern::ic_scale_spectrum(dhat, N, pitch, geom->box, A, c.omega_m, c.h, c.n_s, s); });
    auto derived = [&](const float2* src, int kind, float* dst) {
      stage("spectral factor", s, [&] { return kern::ic_spectral_factor(src, spec, N, pitch, geom->box, kind, s); });
      c2r_real(spec, N, dst, inv_n3, s);
    };
    for (int j = 0; j < 3; ++j) derived(dhat, j, out->psi1 + j * n);
    derived(dhat, 3, r0);  // phi_xx
    derived(dhat, 4, r1);  // phi_yy
    derived(dhat, 5, r2);  // phi_zz
    stage("source", s, [&] { return kern::ic_source_init(r0, r1, r2, n, s); });
    for (int kind = 6; kind < 9; ++kind) {  // phi_xy, phi_xz, phi_yz
      derived(dhat, kind, r1);
      stage("source", s, [&] { return kern::ic_sub_square(r0, r1, n, s); });
    }
    r2c_real(r0, N, dhat, s);  // source spectrum replaces delta_hat
    for (int j = 0; j < 3; ++j) derived(dhat, 9 + j, out->psi2 + j * n);
    const double d1 = host::growth_D1(c, a_init), d2 = host::growth_D2(c, a_init);
    const double E = host::hubble_E(c, a_init), a3 = a_init * a_init * a_init;
    const double f1 = a3 * E * host::growth_dD1(c, a_init), f2 = a3 * E * host::growth_dD2(c, a_init);
    stage("assemble", s, [&] { return kern::ic_assemble(out->pos, out->vel, out->id, out->psi1, out->psi2, N, geom->box, static_cast<float>(d1),
                            static_cast<float>(d2), static_cast<float>(f1), static_cast<float>(f2), s); });
    return finish(flags, s);
  });
}

lpc_status lpc_power_spectrum(const lpc_geometry* geom, const float* pos, int64_t n, double k_max, int32_t n_bins,
                              double* k_mean, double* pk, int64_t* n_modes, void* ws, size_t ws_bytes, void* stream) {
  if (lpc_status st = check_geom_mesh(geom)) return st;
  if (n <= 0 || n > (int64_t(1) << 31) - 1) return fail(LPC_ERR_INVALID_ARG, "n must be in [1, 2^31 - 1]");
  if (!pos || !k_mean || !pk || !n_modes) return fail(LPC_ERR_INVALID_ARG, "NULL array");
  if (n_bins < 1 || n_bins > 2048) return fail(LPC_ERR_INVALID_ARG, "n_bins must be in [1, 2048]");
  if (!(k_max > 0.0) || !std::isfinite(k_max)) return fail(LPC_ERR_INVALID_ARG, "k_max must be positive");
  const Plan p = make_ws_plan(geom->n_mesh, LPC_OP_POWER_SPECTRUM);
  if (lpc_status st = check_ws(ws, ws_bytes, p.total)) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  return guarded([&]() {
    const int nm = geom->n_mesh, pitch = kern::mesh_pitch(nm), nh = nm / 2 + 1;
    const size_t M = static_cast<size_t>(nm) * nm * nm;
    int* flags = reinterpret_cast<int*>(ws);
    uint64_t* dens = reinterpret_cast<uint64_t*>(at(ws, p.dens));
    float2* A = reinterpret_cast<float2*>(at(ws, p.A));
    double* sums = reinterpret_cast<double*>(at(ws, p.bins));
    unsigned long long* counts = reinterpret_cast<unsigned long long*>(sums + 2 * n_bins);
    const double scale = (static_cast<double>(nm) * 65536.0) / geom->box;
    const double mscale = (static_cast<double>(M) / static_cast<double>(n)) * 0x1.0p-48;
    stage("clear flags", s, [&] { return kern::fill_i32(flags, kern::kNumFlags, 0, s); });
    stage("clear bins", s, [&] { return kern::fill_u64(reinterpret_cast<uint64_t*>(sums), static_cast<size_t>(3) * n_bins, s); });
    stage("fill density", s, [&] { return kern::fill_u64(dens, M, s); });
    stage("deposit", s, [&] { return kern::deposit(pos, n, nm, scale, dens, flags, s); });
    stage("fft z r2c", s, [&] { return kern::fft_z_r2c_fixed(dens, nm, mscale, A, pitch, flags, s); });
    stage("fft y", s, [&] { return kern::fft_axis(A, nm, pitch, static_cast<int64_t>(nm) * pitch, nm, nh, 1, 0, false, s); });
    stage("fft x", s, [&] { return kern::fft_axis(A, nm, static_cast<int64_t>(nm) * pitch, pitch, nm, nh, 1, 0, false, s); });
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

lpc_status lpc_fft_r2c(int32_t n, const float* in, float* out_complex, void* ws, size_t ws_bytes, void* stream) {
  if (lpc_status st = check_mesh(n, "n")) return st;
  if (!in || !out_complex) return fail(LPC_ERR_INVALID_ARG, "NULL array");
  const Plan p = make_ws_plan(n, LPC_OP_FFT);
  if (lpc_status st = check_ws(ws, ws_bytes, p.total)) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  return guarded([&]() {
    int* flags = reinterpret_cast<int*>(ws);
    stage("clear flags", s, [&] { return kern::fill_i32(flags, kern::kNumFlags, 0, s); });
    r2c_real(in, n, reinterpret_cast<float2*>(out_complex), s);
    return finish(flags, s);
  });
}

lpc_status lpc_fft_c2r(int32_t n, float* in_complex, float* out, void* ws, size_t ws_bytes, void* stream) {
  if (lpc_status st = check_mesh(n, "n")) return st;
  if (!in_complex || !out) return fail(LPC_ERR_INVALID_ARG, "NULL array");
  const Plan p = make_ws_plan(n, LPC_OP_FFT);
  if (lpc_status st = check_ws(ws, ws_bytes, p.total)) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  return guarded([&]() {
    int* flags = reinterpret_cast<int*>(ws);
    stage("clear flags", s, [&] { return kern::fill_i32(flags, kern::kNumFlags, 0, s); });
    c2r_real(reinterpret_cast<float2*>(in_complex), n, out, 1.0f, s);
    return finish(flags, s);
  });
}

}  // extern "C"
