/*
 * lpc.h -- C ABI of liblpc.so: the particle-mesh COLA time step of L-PICOLA (Howlett, Manera & Percival 2015)
 * on one AMD MI355X (gfx950).
 *
 * The problem statement follows Sec. 3 of the paper: N^3 particles, an Nm^3 mesh, a periodic box of side L (Mpc/h),
 * a flat cosmology and a list of output times. Everything on the hot path runs in hand-written HIP kernels.
 *
 * Conventions shared by every call
 *  - Units: lengths in Mpc/h, time is the scale factor a, H0 = 1. Momenta are p = a^2 dx/dt / H0 in Mpc/h
 *    (peculiar velocity in km/s is 100 p / a).
 *  - Particles are structure-of-arrays in device memory, each vector field as [3][n] floats
 *    (x components, then y, then z). Particle order is preserved by every call; `id` is the lattice index.
 *  - Meshes: node i of an axis sits at i L / Nm. Mesh sizes must factor into 2, 3 and 5, be even, and lie in
 *    [8, 1024]. The initial-condition lattice side N obeys the same rule (its transforms use the same FFT).
 *  - Memory: all device buffers (particles, outputs, workspace) are owned by the caller. The library allocates
 *    no device memory. `ws` is a device buffer of at least lpc_workspace_bytes(geometry, op) bytes, 256-byte
 *    aligned; its contents are scratch and may be overwritten.
 *  - Streams: `stream` is a hipStream_t passed as void* (NULL = the default stream). Every call enqueues its work
 *    on that stream and then waits for it once, to read back the device error flags; on return the outputs are
 *    complete.
 *  - Errors: every call returns an lpc_status; no C++ exception crosses this boundary. lpc_last_error() gives a
 *    human-readable detail of the last failure on the calling thread. On an argument error nothing is enqueued.
 *  - Concurrency: calls that share a workspace must not overlap.
 */
#ifndef LPC_H
#define LPC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  LPC_OK = 0,
  LPC_ERR_INVALID_ARG = -1,      /* null pointer, non-positive size, unordered time list, ... */
  LPC_ERR_UNSUPPORTED_SIZE = -2, /* mesh or lattice size outside what the FFT supports */
  LPC_ERR_WORKSPACE = -3,        /* workspace too small or misaligned */
  LPC_ERR_HIP = -4,              /* a HIP runtime call failed (detail in lpc_last_error) */
  LPC_ERR_FIXED_OVERFLOW = -5,   /* a density cell exceeded the 64-bit fixed-point headroom (>= 2^63) */
  LPC_ERR_NONFINITE = -6,        /* a particle coordinate was NaN/Inf or absurdly far outside the box */
  LPC_ERR_CAPACITY = -7          /* an output buffer was too small (the count needed is reported) */
} lpc_status;

/* Flat LCDM cosmology: Omega_Lambda = 1 - omega_m. The linear spectrum is A k^n_s T_BBKS(k)^2 with shape
 * parameter Gamma = omega_m h, normalised to sigma8 (top-hat, 8 Mpc/h). */
typedef struct {
  double omega_m;
  double h;
  double sigma8;
  double n_s;
} lpc_cosmology;

/* N = n_side particles per side (lattice), Nm = n_mesh cells per side, L = box in Mpc/h. */
typedef struct {
  int32_t n_side;
  int32_t n_mesh;
  double box;
} lpc_geometry;

/* Time stepping (Sec. 2.3). cola: 1 = integrate in the 2LPT frame (Eqs. 17-18), 0 = plain PM (Eqs. 14-15).
 * modified: 1 = the modified kick/drift factors with nLPT (Eq. 19), 0 = the Quinn et al. factors (Eq. 16).
 * deconv_power: divide the force spectrum by the CIC window this many times (0, 1 or 2); default 1. */
typedef struct {
  int32_t cola;
  int32_t modified;
  double n_lpt;
  int32_t deconv_power;
  int32_t reserved; /* must be 0 */
} lpc_stepping;

/* Device structure-of-arrays particle set: pos, vel, psi1, psi2 are float[3][n]; id is int32[n]. */
typedef struct {
  float* pos;
  float* vel;
  float* psi1;
  float* psi2;
  int32_t* id;
  int64_t n;
} lpc_particles;

/* Operation codes for lpc_workspace_bytes. */
enum {
  LPC_OP_INIT_IC = 1,
  LPC_OP_PM_FORCE = 2,
  LPC_OP_COLA_STEP = 3,
  LPC_OP_POWER_SPECTRUM = 4,
  LPC_OP_FFT = 5,
  LPC_OP_BISPECTRUM = 6
};

/* Number of columns of the per-time coefficient table written by lpc_cola_coefficients. */
#define LPC_COEF_COLUMNS 12

/* Workspace bytes needed by operation `op` for this geometry and n_particles particles (0 on an invalid geometry,
 * op or count). PM_FORCE, COLA_STEP, POWER_SPECTRUM and BISPECTRUM need 1 <= n_particles <= 2^31 - 1: their workspace holds
 * tile-sorted copies of the particles (about 16 B per particle for a force or spectrum, 112 B for a COLA run) next
 * to the meshes; INIT_IC and FFT ignore n_particles. */
size_t lpc_workspace_bytes(const lpc_geometry* geom, int32_t op, int64_t n_particles);

/* 2LPT initial conditions at scale factor a_init (Sec. 2.1 Eqs. 5-10; Sec. 5).
 * Draws a unit Gaussian per lattice point from SplitMix64 (Steele, Lea & Flood 2014) in counter mode:
 *   u(c) = ((mix(seed + (c + 1) * 0x9E3779B97F4A7C15) >> 11) + 0.5) 2^-53,
 *   noise(idx) = sqrt(-2 ln u(2 idx)) cos(2 pi u(2 idx + 1)), idx = (i N + j) N + l,
 * scales its Fourier modes by sqrt(P(k) N^3 / L^3) (modes at k = 0 or on a Nyquist plane are zeroed), and solves
 * lap(phi1) = delta_L, lap(phi2) = sum_{i>j} (phi1_ii phi1_jj - phi1_ij^2) spectrally. Outputs (all [3][n], n = N^3):
 *   psi1 = -grad phi1, psi2 = grad phi2 (z = 0 displacements, D1(1) = 1),
 *   pos  = q + D1(a) psi1 + D2(a) psi2 wrapped into [0, L), q = (i + 1/2, j + 1/2, l + 1/2) L / N,
 *   vel  = a^3 E(a) (D1'(a) psi1 + D2'(a) psi2), id = idx.
 * `out->n` must equal N^3. D2 is the Bouchet approximation of Eq. 7. */
lpc_status lpc_init_ic(const lpc_geometry* geom, const lpc_cosmology* cosmo, uint64_t seed, double a_init,
                       const lpc_particles* out, void* ws, size_t ws_bytes, void* stream);

/* Primordial non-Gaussianity in the initial conditions (Sec. 5: local, equilateral, orthogonal or a generic kernel).
 * The Gaussian primordial potential phi is drawn from the same white noise as lpc_init_ic, with power
 * A k^(ns - 4) / alpha0^2 (A the sigma8 amplitude of the linear spectrum, alpha0 = (2/3) (c/H0)^2 g0 / Om, g0 the
 * growth suppression D1(1) / lim_{a->0} D1(a) / a). The non-Gaussian potential is
 *   Phi = phi + f_nl (NL - <NL>),  NL = sum_t c_t D^g_t[(D^a_t phi) (D^b_t phi)],
 * where D^s multiplies Fourier mode k by k^(s (4 - ns) / 3) (k in h/Mpc; |k|^s for a scale-invariant spectrum), so a
 * kernel whose exponents sum to zero per term has the bispectrum of the matching shape in fractional powers of P.
 * The linear density is delta_L(k) = alpha0 k^2 T(k) Phi(k) (f_nl = 0 gives lpc_init_ic's field, to rounding;
 * positive f_nl skews the density positively); the 2LPT construction then proceeds as in lpc_init_ic. */
typedef struct {
  double c; /* coefficient */
  double a; /* D exponents (each within [-4, 4]): inner a and b, outer g */
  double b;
  double g;
} lpc_png_term;

typedef struct {
  double f_nl;
  int32_t n_terms;  /* 1..4 (at most 5 distinct inner exponents in all) */
  int32_t reserved; /* must be 0 */
  lpc_png_term terms[4];
} lpc_png;

enum { LPC_PNG_LOCAL = 0, LPC_PNG_EQUILATERAL = 1, LPC_PNG_ORTHOGONAL = 2 };

/* The kernels of the standard shapes (host only): local NL = phi^2; equilateral (Creminelli et al. 2006)
 * -3 phi^2 + 6 D^-1[(D phi) phi] - 2 D^-2[(D phi)^2]; orthogonal (Senatore et al. 2010)
 * -9 phi^2 + 18 D^-1[(D phi) phi] - 8 D^-2[(D phi)^2]. */
lpc_status lpc_png_preset(int32_t kind, double f_nl, lpc_png* out);

/* lpc_init_ic with the non-Gaussian linear field of `png` (host struct). Workspace: lpc_workspace_bytes(geom,
 * LPC_OP_INIT_IC, 0), as for lpc_init_ic. */
lpc_status lpc_init_ic_png(const lpc_geometry* geom, const lpc_cosmology* cosmo, uint64_t seed, double a_init,
                           const lpc_png* png, const lpc_particles* out, void* ws, size_t ws_bytes, void* stream);

/* The particle-mesh force of Sec. 2.4 (Eqs. 20-21) at positions pos[3][n]:
 *   particles sorted by mesh tile (16 x 8 x 32 cells along x, y, z) into the workspace (the single-GPU counterpart
 *   of moving particles to the process that owns their slab, Sec. 4.4), fixed-point CIC deposit by one workgroup
 *   per tile
 *   (16 fractional bits per axis, int64 counts, each particle adds exactly 2^48),
 *   delta = C (Nm^3 / n) 2^-48 - 1, forward r2c FFT, g_hat_j = i k_j (-1/k^2) delta_hat / W^p
 *   (W = prod sinc^2(pi n_d / Nm), p = step->deconv_power, zero at k = 0 and on the Nyquist plane of axis j),
 *   three c2r FFTs, CIC gather with the deposit's own fixed-point fractions.
 * grad_out[3][n] receives grad(psi) with lap(psi) = delta (Mpc/h). density_fixed_out, if not NULL, receives the
 * int64 counts C[Nm][Nm][Nm] (x-major). Only step->deconv_power is read from `step`. geom->n_side is not used. */
lpc_status lpc_pm_force(const lpc_geometry* geom, const lpc_stepping* step, const float* pos, int64_t n,
                        float* grad_out, int64_t* density_fixed_out, void* ws, size_t ws_bytes, void* stream);

/* Bytes of the static device scratch behind lpc_pm_force_noalloc (64 MiB per GPU, held from the library's load until
 * the process ends). */
#define LPC_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)

/* lpc_pm_force without a workspace argument and without any device allocation, for callers that cannot allocate:
 * code under HIP graph capture, serving loops that must not call hipMalloc, harnesses that forbid it. The workspace
 * is a static device array of LPC_NOALLOC_SCRATCH_BYTES inside the library, one per GPU, looked up for the current
 * device (the stream must belong to it). Arguments, outputs and results are those of lpc_pm_force (same kernels, the
 * same bits). A geometry and count whose lpc_workspace_bytes(geom, LPC_OP_PM_FORCE, n) exceeds the scratch (for
 * example a 128^3 mesh with more than about 400k particles, or a 96^3 mesh with more than about 1.8M) is rejected with
 * LPC_ERR_WORKSPACE before anything is enqueued. Every call on one GPU shares that GPU's scratch: calls that overlap
 * on one GPU (two streams, two threads) race and must be serialised by the caller. The scratch keeps the last
 * call's contents; everything a call needs cleared it clears itself. */
lpc_status lpc_pm_force_noalloc(const lpc_geometry* geom, const lpc_stepping* step, const float* pos, int64_t n,
                                float* grad_out, int64_t* density_fixed_out, void* stream);

/* Advance particles from a_list[0] to a_list[n_a - 1] with the kick-drift-kick COLA integrator (Sec. 2.3):
 * frame momentum removed at a_0 (Sec. 2.3), then for i = 0..n_a-1: force at a_i, kick a_{i-1/2} -> a_{i+1/2}
 * (midpoints; a_{-1/2} = a_0, a_{N+1/2} = a_N), drift a_i -> a_{i+1} for i < n_a - 1; frame momentum added back at
 * the last time. inout->vel holds the Eulerian momentum at a_list[0] on entry and at a_list[n_a-1] on exit.
 * a_list is a host array, strictly increasing, positive, n_a >= 2. With cola = 0, psi1 and psi2 are not read.
 * The run works on tile-sorted copies of the particles in the workspace (re-sorted before every force evaluation)
 * and writes pos and vel back in the caller's order at the end; psi1, psi2 and id are not modified. */
lpc_status lpc_cola_step(const lpc_geometry* geom, const lpc_cosmology* cosmo, const lpc_stepping* step,
                         const double* a_list, int32_t n_a, const lpc_particles* inout, void* ws, size_t ws_bytes,
                         void* stream);

/* ---------------------------------------------------------------------------------------------------------------
 * On-the-fly lightcone (Sec. 6.1) with box replicates (Sec. 6.2).
 *
 * Speed of light over H0 in Mpc/h (H0 = 100 h km/s/Mpc): the unit of comoving distance. */
#define LPC_C_OVER_H0 2997.92458

/* Comoving distance R_L(a) = (c / H0) int_a^1 da' / (a'^2 E(a')) in Mpc/h, the radius of the past lightcone of an
 * observer at a = 1 (Sec. 6), at host scale factors a[m] in (0, 1] into host r[m] (host only). */
lpc_status lpc_comoving_distance(const lpc_cosmology* cosmo, const double* a, int32_t m, double* r);

/* One particle image leaving the lightcone. */
typedef struct {
  float pos[3];      /* comoving position at a (Mpc/h) in the replicated volume: box position + L (i, j, k) */
  float vel[3];      /* momentum p = a^2 dx/dt / H0 (Mpc/h) at the drift's midpoint a_{i+1/2} (not interpolated) */
  float a;           /* the scale factor at which the image left the lightcone */
  int32_t index;     /* the particle's index in the caller's arrays */
  int32_t replicate; /* ((i - rep_lo[0]) n_y + (j - rep_lo[1])) n_z + (k - rep_lo[2]), n_d = rep_hi[d] - rep_lo[d] + 1 */
  int32_t reserved;  /* 0 */
} lpc_lightcone_record;

/* The lightcone of a run: an observer at `origin` (Mpc/h, in the box frame), active on every drift that starts at
 * a >= a_start; the box repeated on the offsets L (i, j, k), rep_lo[d] <= i, j, k <= rep_hi[d] (all 0: the box
 * alone; at most 32768 replicates, each index within +-1024); `records` is a DEVICE array of `capacity` records
 * (caller-owned; NULL allowed when capacity is 0). */
typedef struct {
  double origin[3];
  double a_start;
  int32_t rep_lo[3];
  int32_t rep_hi[3];
  lpc_lightcone_record* records;
  int64_t capacity;
} lpc_lightcone;

/* lpc_cola_step (same arguments, workspace lpc_workspace_bytes(geom, LPC_OP_COLA_STEP, n), same final particles) with
 * the lightcone drift of Sec. 6.1. In each lightcone drift a_i -> a_{i+1} every particle image (the wrapped position
 * plus a replicate offset, drifted without wrapping) is tested: it leaves the lightcone when R_p(a_i) <= R_L(a_i)
 * and R_p(a_{i+1}) > R_L(a_{i+1}), R_p being its distance to the observer. Its crossing time comes from the linear
 * interpolation of R_p and R_L between a_i and a_{i+1} (the interpolation equation of Sec. 6.1), its position from
 * the drift (Sec. 2.3) from a_i to that time, its momentum is the one at a_{i+1/2} plus, for COLA, the frame momentum
 * a^3 E (D1' psi1 + D2' psi2) there. Replicates whose closest point lies beyond R_L(a_i) are skipped for that drift and
 * all later ones (Sec. 6.2.3); each workgroup also skips images its particles' bounding boxes cannot cross. Records
 * are appended in no fixed order; *n_records (host) receives their number. When it exceeds lc->capacity the records
 * past the capacity are dropped and LPC_ERR_CAPACITY is returned (the particles are still advanced). a_list ends at
 * a <= 1 and holds at most 1000 times. */
lpc_status lpc_cola_step_lightcone(const lpc_geometry* geom, const lpc_cosmology* cosmo, const lpc_stepping* step,
                                   const double* a_list, int32_t n_a, const lpc_particles* inout,
                                   const lpc_lightcone* lc, int64_t* n_records, void* ws, size_t ws_bytes,
                                   void* stream);

/* One box of a batched run: its geometry (n_side unused) and its device particles (pos, vel, psi1, psi2). */
typedef struct {
  lpc_geometry geom;
  lpc_particles particles;
} lpc_batch_entry;

/* Workspace bytes of lpc_cola_step_batched for these n_real entries (0 if any mesh size is unsupported):
 * flags, the job tables and, per entry in order, its own int64/force mesh and three half-spectrum meshes. */
size_t lpc_workspace_bytes_batched(const lpc_batch_entry* entries, int32_t n_real);

/* The run of lpc_cola_step (Sec. 2.3 integrator, Sec. 2.4 force) for n_real independent boxes at once: the many
 * independent realisations (mocks) that a covariance estimate needs (Sec. 1). The boxes may differ in mesh
 * size, box side and particle count; they share the cosmology, the stepping options and the time list. Every stage
 * (deposit, each FFT pass, Poisson, gather/kick/drift) is ONE launch over all boxes, whose workgroups take the
 * (box, tile) items of a work table; the results equal n_real separate lpc_cola_step calls bit for bit.
 * `entries` is a host array of 1..4096 entries; `ws` holds lpc_workspace_bytes_batched(entries, n_real) bytes.
 * The enqueued kernels are recorded once into a HIP graph and replayed while every argument (entries, cosmology,
 * stepping, time list, workspace pointer) repeats; lpc_graph_enable(0) launches them directly instead. The graph
 * cache is process-wide: batched calls must not overlap across threads. */
lpc_status lpc_cola_step_batched(const lpc_batch_entry* entries, int32_t n_real, const lpc_cosmology* cosmo,
                                 const lpc_stepping* step, const double* a_list, int32_t n_a, void* ws,
                                 size_t ws_bytes, void* stream);

/* Switch graph replay of lpc_cola_step_batched on (default) or off. Profiling (lpc_profile_enable) also turns it
 * off, since per-stage events are recorded between launches. */
lpc_status lpc_graph_enable(int32_t on);

/* Binned power spectrum of the particles (periodic box; Sec. 7.1): fixed-point CIC deposit on the Nm mesh,
 * r2c FFT, P = L^3 |delta_hat|^2 / (Nm^6 W^2) (one CIC window removed in amplitude), bins [b dk, (b+1) dk) of |k|
 * with dk = k_max / n_bins, the k = 0 mode excluded, half-spectrum modes with 0 < n_z < Nm/2 counted twice.
 * No shot-noise subtraction. k_mean, pk (double) and n_modes (int64) are HOST arrays of n_bins; empty bins give
 * NaN for k_mean and pk. */
lpc_status lpc_power_spectrum(const lpc_geometry* geom, const float* pos, int64_t n, double k_max, int32_t n_bins,
                              double* k_mean, double* pk, int64_t* n_modes, void* ws, size_t ws_bytes, void* stream);

/* Reduced bispectrum Q(k1, k2, k3) of the particles (periodic box; the three-point statistic of Sec. 7.2), by the
 * FFT shell estimator: the density spectrum of lpc_power_spectrum with one CIC window removed (delta_hat / W); shell
 * b = {modes with k_b - dk/2 <= |k| < k_b + dk/2}; for each triangle, F_i(x) = sum over shell i of delta_hat e^{ikx}
 * and I_i(x) = sum over shell i of e^{ikx} (inverse transforms), then
 *   B = L^6 / Nm^9 * sum_x F1 F2 F3 / sum_x I1 I2 I3   (the mean of delta_hat1 delta_hat2 delta_hat3 over the closed
 *       triangles n1 + n2 + n3 = 0 with n_i in shell i, in continuous normalisation),
 *   P_i = L^3 / Nm^6 * mean over shell i of |delta_hat / W|^2,   Q = B / (P1 P2 + P2 P3 + P3 P1).
 * No shot-noise subtraction. k123 (HOST, [m][3], h/Mpc, each > 0) are the shell centres of m <= 256 triangles;
 * B and Q (HOST, [m]) receive the results (NaN where no triangle closes: sum_x I1 I2 I3, which is Nm^3 times the
 * number of closed triangles, below Nm^3 / 2), P (HOST, [m][3], or NULL) the shell
 * powers. Sums are FP64, reduced in a fixed order (bitwise repeatable). Workspace: lpc_workspace_bytes(geom,
 * LPC_OP_BISPECTRUM, n), geom->n_mesh the estimator mesh. */
lpc_status lpc_bispectrum(const lpc_geometry* geom, const float* pos, int64_t n, const double* k123, int32_t m,
                          double dk, double* B, double* Q, double* P, void* ws, size_t ws_bytes, void* stream);

/* The FP64 per-time coefficient table of one lpc_cola_step call (host only; for checking and inspection).
 * out[n_a][LPC_COEF_COLUMNS] row i: a_i, D1, D2, dD1/da, dD2/da, E, K_i (kick factor), Q_i (drift factor, 0 in the
 * last row), D1(a_{i+1}) - D1(a_i), D2(a_{i+1}) - D2(a_i) (0 in the last row), a^3 E D1', a^3 E D2'. */
lpc_status lpc_cola_coefficients(const lpc_cosmology* cosmo, const lpc_stepping* step, const double* a_list,
                                 int32_t n_a, double* out);

/* Linear P(k) of the cosmology at host wavenumbers k[m] (h/Mpc) into host pk[m] (host only). */
lpc_status lpc_linear_power(const lpc_cosmology* cosmo, const double* k, int32_t m, double* pk);

/* Unnormalised forward r2c 3-D FFT of a real n^3 device mesh (x-major) into a complex half spectrum with
 * row pitch lpc_fft_pitch(n) complex values: out[(kx * n + ky) * pitch + kz], kz = 0..n/2.
 * X(k) = sum_x f(x) exp(-2 pi i k.x / n). (The same kernels as the force path; exposed for testing.) */
lpc_status lpc_fft_r2c(int32_t n, const float* in, float* out_complex, void* ws, size_t ws_bytes, void* stream);

/* Unnormalised inverse c2r 3-D FFT: f(x) = sum_k X(k) exp(+2 pi i k.x / n) over the Hermitian-completed spectrum.
 * `in_complex` (pitch lpc_fft_pitch(n)) is overwritten. */
lpc_status lpc_fft_c2r(int32_t n, float* in_complex, float* out, void* ws, size_t ws_bytes, void* stream);

/* Row pitch, in complex values, of the half-spectrum layout used by lpc_fft_r2c / lpc_fft_c2r. */
int32_t lpc_fft_pitch(int32_t n);

/* FFT tile shape of one mesh size (measurement and tuning plumbing; the transforms' results do not depend on it).
 * Each pass of a 3-D transform stages a tile of independent 1-D transforms through LDS; these are the tile widths.
 *   z_rows:       rows per tile of the forward z (r2c) pass and of single-spectrum inverse z passes: 8, 16 or 32
 *   axis_cols:    columns per tile of the strided y and x passes (forward and inverse): 8, 16 or 32
 *   poisson_cols: columns per tile of the force path's fused x + Poisson pass: 4, 8 or 16
 *   c2r_rows:     rows per tile of the force path's three-component inverse z pass: 4, 8 or 16
 * A width fits mesh size n when its tile's loads and FFT stages fit one 512-thread workgroup and its LDS is at most
 * 160 KiB. A batched call uses, per pass, the smallest width over its boxes. */
typedef struct {
  int32_t z_rows;
  int32_t axis_cols;
  int32_t poisson_cols;
  int32_t c2r_rows;
} lpc_fft_tiling;

/* The built-in tiling of mesh size n (the widest widths that fit, with the fused pass at most 16 and 8 above
 * n = 512): host only. LPC_ERR_UNSUPPORTED_SIZE for a mesh size the FFTs do not take. */
lpc_status lpc_fft_tiling_default(int32_t n_mesh, lpc_fft_tiling* out);
/* The tiling in effect for mesh size n: the override set by lpc_fft_tiling_set, else the built-in one. */
lpc_status lpc_fft_tiling_get(int32_t n_mesh, lpc_fft_tiling* out);
/* Override the tiling of mesh size n for every later call of this process (t = NULL removes the override).
 * LPC_ERR_INVALID_ARG, with the field named in lpc_last_error(), if a width is not an instantiated one or does not
 * fit n; nothing changes then. Process-wide state, guarded by a mutex; a recorded batched graph is re-recorded on its
 * next call. An autotuner (paper_1506_03737_amd/autotune.py) measures the widths per mesh size and sets them here. */
lpc_status lpc_fft_tiling_set(int32_t n_mesh, const lpc_fft_tiling* t);
/* Remove every override. */
lpc_status lpc_fft_tiling_reset(void);

/* ---------------------------------------------------------------------------------------------------------------
 * Learned displacement correction (not in the paper: a learned stand-in for the small-scale accuracy that a finer PM
 * mesh buys, Sec. 2.4). A coarse run (Nm = N) is corrected toward a fine run (Nm = 3N) by a 3-D convolutional
 * network on the N^3 particle lattice, trained only on pairs of runs of this library.
 *
 * Grid: voxel v = (i N + j) N + l is the lattice site of particle id v. Input grid: FP32 [N^3][6]: channels 0..2
 * the particle's minimal-image displacement from its lattice point q = (i + 1/2, j + 1/2, l + 1/2) L / N, channels
 * 3..5 its first-order 2LPT displacement Psi1 (Sec. 2.1), both in units of L / N. Output: FP32 [N^3][3], the
 * residual displacement (same units) added to the coarse positions.
 * Network (3^3 convolutions with periodic wrap; "down" = 2^3 stride-2 convolution, "up" = 2^3 stride-2 transposed
 * convolution; every layer but the last followed by leaky ReLU, slope 0.1):
 *   a0 = conv(in: 6 -> 16); s0 = conv(a0: 16 -> 16); a1 = down(s0: 16 -> 32) at N/2; s1 = conv(a1: 32 -> 32);
 *   a2 = down(s1: 32 -> 64) at N/4; b2 = conv(a2: 64 -> 64); u1 = up(b2: 64 -> 32) at N/2;
 *   c1 = conv([u1, s1]: 64 -> 32); u0 = up(c1: 32 -> 16) at N; c0 = conv([u0, s0]: 32 -> 16); out = conv(c0: 16 -> 3).
 * Parameters: one FP32 vector (lpc_net_param_count() values); per layer in the order above, W[Cout][taps][Cin] with
 * taps x-major (t = (tx K + ty) K + tz, K = 3 or 2), then b[Cout]. Loss: mean over voxels and channels of
 * (out - target)^2. Precision: activations and their gradients BF16, 3^3 convolutions (forward and data gradient) and
 * the forward down/up layers on BF16 MFMA with FP32 accumulation (weights rounded to BF16), weight gradients FP32 sums
 * of BF16 products, master weights and Adam state FP32. n_side must be a multiple of 4 in [8, 512]. Device buffers
 * are caller-owned; device params must be 16-byte aligned (LPC_ERR_INVALID_ARG otherwise); ws holds
 * lpc_net_workspace_bytes() bytes (256-byte aligned) and is scratch for every call below. */
int64_t lpc_net_param_count(void);

/* Host-side initialisation of params[lpc_net_param_count()] (host FP32): W uniform in +-sqrt(6 / (taps Cin))
 * (0.1 x that for the last layer), b = 0, from SplitMix64 seeded with `seed`. */
lpc_status lpc_net_init(float* params, uint64_t seed);

size_t lpc_net_workspace_bytes(int32_t n_side);

/* Input grid (psi1 given, ref_pos NULL: out is [N^3][6]) or target grid (ref_pos given, psi1 NULL: out is [N^3][3])
 * of N^3 particles pos[3][n] with lattice ids id[n]: out[id][d] = minimal image (pos - base) / (L / N) with base the
 * lattice point of id, or ref_pos[3][n] (the same particles in another run: target = fine - coarse); and
 * out[id][3 + d] = psi1[d][p] / (L / N). With neither, out is the displacement alone ([N^3][3]). An id outside
 * [0, N^3) gives LPC_ERR_INVALID_ARG. */
lpc_status lpc_net_features(const lpc_geometry* geom, const float* pos, const int32_t* id, int64_t n,
                            const float* ref_pos, const float* psi1, float* out, void* ws, size_t ws_bytes,
                            void* stream);

/* out[N^3][3] = network(feat[N^3][6]) with device params. */
lpc_status lpc_net_forward(int32_t n_side, const float* params, const float* feat, float* out, void* ws,
                           size_t ws_bytes, void* stream);

/* Loss of the network on one sample and its gradient grad[lpc_net_param_count()] (device, overwritten) by
 * backpropagation; *loss (host) receives the loss. */
lpc_status lpc_net_loss_grad(int32_t n_side, const float* params, const float* feat, const float* target,
                             float* grad, double* loss, void* ws, size_t ws_bytes, void* stream);

/* One Adam step (Kingma & Ba 2015; beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected, step counts from 1) on the
 * device vectors params, m, v with gradient grad. */
lpc_status lpc_net_adam(float* params, float* m, float* v, const float* grad, int64_t step, float lr, void* stream);

/* Scales the network's output in place: the output layer (the last, linear layer: its weights and biases) of the
 * device parameter vector params is multiplied by gain, so network(x) becomes gain network(x) up to the BF16 rounding
 * of the scaled weights. Used to calibrate a trained correction against the statistic it is evaluated by (the trainer
 * picks gain on held-out pairs). Asynchronous on `stream`; LPC_ERR_INVALID_ARG for a NULL or misaligned params or a
 * non-finite gain. */
lpc_status lpc_net_scale_output(float* params, float gain, void* stream);

/* Training-data augmentation: out = the k-th (0..47) symmetry of the periodic cube applied to a lattice field of
 * 3-vectors, in and out FP32 [n_side^3][channels] (channels = 3 m: m vectors per site, e.g. 6 for an input grid, 3
 * for a target grid; device pointers that must not overlap). k = 8 p + f maps space by x'_d = x_{perm[d]} with perm
 * the p-th of (0 1 2), (0 2 1), (1 0 2), (1 2 0), (2 0 1), (2 1 0), then reflects axis d (x'_d -> L - x'_d, lattice
 * site i -> n_side - 1 - i) for each bit d of f; a vector v at site u moves to the image site as v'_d = +-v_{perm[d]}
 * (minus on a reflected axis). The equations of motion are invariant under these maps, so a pair of runs maps to
 * a valid pair. Asynchronous on `stream`; LPC_ERR_INVALID_ARG for k, channels or n_side out of range, or overlap. */
lpc_status lpc_net_symmetry(int32_t n_side, int32_t k, int32_t channels, const float* in, float* out, void* stream);

/* Corrects a coarse run in place: pos += network(input grid(pos, psi1, id)) L / N, wrapped into [0, L). inout->n must
 * be n_side^3 (one particle per lattice site); only pos, psi1 and id are used. */
lpc_status lpc_net_apply(const lpc_geometry* geom, const float* params, const lpc_particles* inout, void* ws,
                         size_t ws_bytes, void* stream);

/* Per-stage profiling (measurement plumbing, not part of the method). When enabled, every kernel
 * launch of the entry points above is bracketed by HIP events on the call's stream; the durations are read after the
 * call's final synchronisation and accumulated per stage name ("deposit", "fft y inv", ...). Process-wide state,
 * not thread safe. lpc_profile_get returns stage i's name (valid until lpc_profile_reset), its launch count and its
 * total milliseconds. */
lpc_status lpc_profile_enable(int32_t on);
lpc_status lpc_profile_reset(void);
int32_t lpc_profile_count(void);
lpc_status lpc_profile_get(int32_t i, const char** name, int64_t* launches, double* total_ms);

const char* lpc_status_string(lpc_status s);
const char* lpc_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* LPC_H */
