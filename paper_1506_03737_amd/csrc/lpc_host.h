// Internal host-side declarations of liblpc (not part of the C ABI).
#pragma once

#include <cstddef>
#include <cstdint>

namespace lpc {
namespace host {

struct Cosmo {
  double omega_m, h, sigma8, n_s;
};

// Column indices of the per-time coefficient table (same order as the ABI documents).
enum { kA = 0, kD1, kD2, kdD1, kdD2, kE, kK, kQ, kDD1, kDD2, kF1, kF2, kCoefColumns };

double hubble_E(const Cosmo& c, double a);
double growth_D1(const Cosmo& c, double a);
double growth_dD1(const Cosmo& c, double a);
double growth_D2(const Cosmo& c, double a);
double growth_dD2(const Cosmo& c, double a);
double kick_factor(const Cosmo& c, double a_lo, double a_i, double a_hi, bool modified, double n_lpt);
double drift_factor(const Cosmo& c, double a_i, double a_ip1, bool modified, double n_lpt);
// The drift factor from a_i to a within the step a_i -> a_{i+1} (the modified form keeps the step's normalisation
// u(a_{i+1/2})); drift_factor(a_i, a_{i+1}) is the case a = a_{i+1}.
double partial_drift_factor(const Cosmo& c, double a_i, double a, double a_ip1, bool modified, double n_lpt);
// Comoving distance to scale factor a, (c / H0) int_a^1 da / (a^2 E), in Mpc/h.
constexpr double kCOverH0 = 2997.92458;
double comoving_distance(const Cosmo& c, double a);
// g0 = D1(1) / lim_{a->0} D1(a) / a = (5/2) Om int_0^1 da / (a E)^3: the growth suppression of D1(1) = 1.
double growth_suppression(const Cosmo& c);
void coefficient_table(const Cosmo& c, bool modified, double n_lpt, const double* a, int n, double* out);
double pk_amplitude(const Cosmo& c);
double linear_pk(const Cosmo& c, double amplitude, double k);

}  // namespace host
}  // namespace lpc
