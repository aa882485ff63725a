// Host-side FP64 cosmology for liblpc: growth factors, the KDK factors of Sec. 2.3 and the BBKS linear spectrum.
//
// Quadratures are fixed-order Gauss-Legendre rules (nodes by Newton iteration on the Legendre recurrence). The
// equations follow Sec. 2.1 (Eq. 7, Bouchet D2) and Sec. 2.3 (Eq. 16 standard factors, Eq. 19 modified factors) of
// Howlett, Manera & Percival (2015), with these readings:
//  - D1 is the growing mode E(a) int_0^a da' / (a' E)^3, normalised to D1(1) = 1;
//  - with p = a^2 dx/dt / H0: dp/da = F / (a^2 E) and dx/da = p / (a^3 E), so the standard kick factor is
//    int da / (a^2 E) and the modified one [u(a+) - u(a-)] / (u'(a_i) a_i^2 E(a_i)), u = a^nLPT; the drift factors
//    are int da / (a^3 E) and int u / (a^3 E) da / u(a_{i+1/2});
//  - the frame momentum is a^3 E (D1' psi1 + D2' psi2).
#include <cmath>
#include <vector>

#include "lpc_host.h"

namespace lpc {
namespace host {

namespace {

struct GaussLegendre {
  std::vector<double> x, w;  // nodes and weights on [-1, 1]
  explicit GaussLegendre(int n) : x(n), w(n) {
    for (int i = 0; i < (n + 1) / 2; ++i) {
      double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
      double dp = 0.0;
      for (int it = 0; it < 100; ++it) {
        double p0 = 1.0, p1 = 0.0;
        for (int j = 1; j <= n; ++j) {  // P_j(z) = ((2j-1) z P_{j-1} - (j-1) P_{j-2}) / j
          double p2 = p1;
          p1 = p0;
          p0 = ((2.0 * j - 1.0) * z * p1 - (j - 1.0) * p2) / j;
        }
        dp = n * (z * p0 - p1) / (z * z - 1.0);
        double dz = p0 / dp;
        z -= dz;
        if (std::fabs(dz) < 1e-16) break;
      }
      x[i] = -z;
      x[n - 1 - i] = z;
      w[i] = w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
  }
};

const GaussLegendre& gl64() {
  static const GaussLegendre g(64);
  return g;
}

template <class F>
double integrate(F f, double lo, double hi, int pieces = 1) {
  const GaussLegendre& g = gl64();
  double total = 0.0, h = (hi - lo) / pieces;
  for (int p = 0; p < pieces; ++p) {
    double a = lo + p * h, b = a + h, c = 0.5 * (a + b), r = 0.5 * (b - a), s = 0.0;
    for (size_t i = 0; i < g.x.size(); ++i) s += g.w[i] * f(c + r * g.x[i]);
    total += r * s;
  }
  return total;
}

}  // namespace

double hubble_E(const Cosmo& c, double a) { return std::sqrt(c.omega_m / (a * a * a) + (1.0 - c.omega_m)); }

// int_0^a da' / (a' E(a'))^3 with a' = t^2: the integrand 2 t^4 (Om + OL t^6)^(-3/2) is smooth at t = 0.
static double heath(const Cosmo& c, double a) {
  const double om = c.omega_m, ol = 1.0 - c.omega_m;
  auto f = [om, ol](double t) {
    double t2 = t * t;
    double s = om + ol * t2 * t2 * t2;
    return 2.0 * t2 * t2 / (s * std::sqrt(s));
  };
  return integrate(f, 0.0, std::sqrt(a), 4);
}

static double d1_norm(const Cosmo& c) { return hubble_E(c, 1.0) * heath(c, 1.0); }

double growth_D1(const Cosmo& c, double a) { return hubble_E(c, a) * heath(c, a) / d1_norm(c); }

// Early on E ~ sqrt(Om) a^(-3/2) and the integral ~ (2/5) a^(5/2) / Om^(3/2), so D1(a) -> (2/5) a / (Om norm).
double growth_suppression(const Cosmo& c) { return 2.5 * c.omega_m * d1_norm(c); }

double growth_dD1(const Cosmo& c, double a) {
  const double E = hubble_E(c, a);
  const double dE = -1.5 * c.omega_m / (a * a * a * a * E);
  const double norm = d1_norm(c);
  return dE / E * (E * heath(c, a) / norm) + 1.0 / (a * a * a * E * E * norm);
}

static double omega_m_a(const Cosmo& c, double a) {
  return c.omega_m / (c.omega_m + (1.0 - c.omega_m) * a * a * a);
}

double growth_D2(const Cosmo& c, double a) {
  const double d1 = growth_D1(c, a);
  return -3.0 / 7.0 * d1 * d1 * std::pow(omega_m_a(c, a), -1.0 / 143.0);
}

double growth_dD2(const Cosmo& c, double a) {
  const double d1 = growth_D1(c, a), dd1 = growth_dD1(c, a), om = omega_m_a(c, a);
  const double g = std::pow(om, -1.0 / 143.0);
  const double dg = (-1.0 / 143.0) * g / om * (-3.0 * om * (1.0 - om) / a);
  return -3.0 / 7.0 * (2.0 * d1 * dd1 * g + d1 * d1 * dg);
}

double kick_factor(const Cosmo& c, double a_lo, double a_i, double a_hi, bool modified, double n_lpt) {
  if (modified) {
    const double du = n_lpt * std::pow(a_i, n_lpt - 1.0);
    return (std::pow(a_hi, n_lpt) - std::pow(a_lo, n_lpt)) / (du * a_i * a_i * hubble_E(c, a_i));
  }
  if (a_hi == a_lo) return 0.0;
  return integrate([&c](double a) { return 1.0 / (a * a * hubble_E(c, a)); }, a_lo, a_hi);
}

double partial_drift_factor(const Cosmo& c, double a_i, double a_end, double a_ip1, bool modified, double n_lpt) {
  if (a_end == a_i) return 0.0;
  if (modified) {
    const double mid = 0.5 * (a_i + a_ip1);
    const double v =
        integrate([&c, n_lpt](double a) { return std::pow(a, n_lpt) / (a * a * a * hubble_E(c, a)); }, a_i, a_end);
    return v / std::pow(mid, n_lpt);
  }
  return integrate([&c](double a) { return 1.0 / (a * a * a * hubble_E(c, a)); }, a_i, a_end);
}

double drift_factor(const Cosmo& c, double a_i, double a_ip1, bool modified, double n_lpt) {
  return partial_drift_factor(c, a_i, a_ip1, a_ip1, modified, n_lpt);
}

// 1 / (a^2 E) = a^(-1/2) / sqrt(Om + OL a^3); with a = s^2 (da = 2 s ds) the integrand becomes
// 2 / sqrt(Om + OL s^6), smooth down to a = 0.
double comoving_distance(const Cosmo& c, double a) {
  const double om = c.omega_m, ol = 1.0 - c.omega_m;
  auto f = [om, ol](double s) {
    const double s2 = s * s;
    return 2.0 / std::sqrt(om + ol * s2 * s2 * s2);
  };
  return kCOverH0 * integrate(f, std::sqrt(a), 1.0, 4);
}

void coefficient_table(const Cosmo& c, bool modified, double n_lpt, const double* a, int n, double* out) {
  for (int i = 0; i < n; ++i) {
    const double ai = a[i];
    const double lo = (i == 0) ? a[0] : 0.5 * (a[i - 1] + a[i]);
    const double hi = (i == n - 1) ? a[n - 1] : 0.5 * (a[i] + a[i + 1]);
    const double d1 = growth_D1(c, ai), d2 = growth_D2(c, ai);
    const double dd1 = growth_dD1(c, ai), dd2 = growth_dD2(c, ai), E = hubble_E(c, ai);
    double* row = out + static_cast<size_t>(i) * kCoefColumns;
    row[kA] = ai;
    row[kD1] = d1;
    row[kD2] = d2;
    row[kdD1] = dd1;
    row[kdD2] = dd2;
    row[kE] = E;
    row[kK] = kick_factor(c, lo, ai, hi, modified, n_lpt);
    if (i + 1 < n) {
      row[kQ] = drift_factor(c, ai, a[i + 1], modified, n_lpt);
      row[kDD1] = growth_D1(c, a[i + 1]) - d1;
      row[kDD2] = growth_D2(c, a[i + 1]) - d2;
    } else {
      row[kQ] = row[kDD1] = row[kDD2] = 0.0;
    }
    row[kF1] = ai * ai * ai * E * dd1;
    row[kF2] = ai * ai * ai * E * dd2;
  }
}

// BBKS transfer function (Bardeen et al. 1986), q = k / (Om h), k in h/Mpc.
static double bbks(const Cosmo& c, double k) {
  const double q = k / (c.omega_m * c.h);
  const double x = 2.34 * q;
  const double a = 16.1 * q, b = 5.46 * q, d = 6.71 * q;
  const double poly = 1.0 + 3.89 * q + a * a + b * b * b + d * d * d * d;
  return std::log1p(x) / x / std::sqrt(std::sqrt(poly));
}

static double tophat(double x) {
  if (std::fabs(x) < 1e-3) return 1.0 - x * x / 10.0;
  return 3.0 * (std::sin(x) - x * std::cos(x)) / (x * x * x);
}

double pk_amplitude(const Cosmo& c) {
  // sigma(8)^2 = (1/(2 pi^2)) int k^3 P W^2 dln k over ln k in [ln 1e-7, ln 1e3]
  auto f = [&c](double lnk) {
    const double k = std::exp(lnk);
    const double t = bbks(c, k), w = tophat(8.0 * k);
    return k * k * k * std::pow(k, c.n_s) * t * t * w * w;
  };
  const double s2 = integrate(f, std::log(1e-7), std::log(1e3), 400) / (2.0 * M_PI * M_PI);
  return c.sigma8 * c.sigma8 / s2;
}

double linear_pk(const Cosmo& c, double amplitude, double k) {
  if (k <= 0.0) return 0.0;
  const double t = bbks(c, k);
  return amplitude * std::pow(k, c.n_s) * t * t;
}

}  // namespace host
}  // namespace lpc
