// hcao_host_tables.cpp -- host-side tables of the step (see hcao_host_tables.h).
//
// Sources: level ladders, Eq. energy-AHO and Eq. energy-SHO (Sec. "The
// polyatomic HCAO model"); the forward probability, its Whitten-Rabinovich
// density of states and the equilibrium constant, Sec. "Recombination
// reactions" with the readings of the determinism specification (regularized
// upper incomplete gamma, N_samp energies, zero-point energy E_z, log base
// 10, K_eq from translational and vibrational partition functions, k_f as the
// forward probability times the Maxwellian A-M collision rate).
#include "hcao_host_tables.h"

#include <algorithm>
#include <cmath>
#include <cstring>

namespace hcao {
namespace host {
namespace {

constexpr double kPlanck = 6.62607015e-34;  // [J s]
constexpr double kLight = 299792458.0;      // [m/s]
constexpr double kBoltzmann = 1.380649e-23;  // [J/K]
constexpr double kPiHost = 3.141592653589793;
constexpr uint32_t kLadderMax = 1024;

// Maxwellian mean of the VHS cross-section times speed of a pair with mean
// diameter d, exponent w, reference temperature tr and reduced mass mr:
// ((2 d^2) sqrt(((2 pi) k tr) / mr)) (t / tr)^(1 - w).
double maxwell_sigma_g(double d, double w, double tr, double mr, double t) {
  const double front = 2.0 * (d * d);
  const double speed = std::sqrt(((2.0 * kPiHost) * kBoltzmann * tr) / mr);
  return front * speed * std::pow(t / tr, 1.0 - w);
}

// Boltzmann mean of e_i = E_i - E_0 over a ladder with weights exp(-x e_i)
// (x = 1 / kT, or beta), summed in ascending order
double ladder_mean(const std::vector<double> &L, double x, bool beta_form) {
  double top = 0.0, bottom = 0.0;
  for (double level : L) {
    const double e = level - L[0];
    const double w = beta_form ? std::exp(-(x * e)) : std::exp(-e / x);
    top = top + e * w;
    bottom = bottom + w;
  }
  return top / bottom;
}

}  // namespace

const char *morse_ladder(double we, double xe, double &de, std::vector<double> &levels) {
  levels.clear();
  if (!(we > 0.0) || !(xe >= 0.0)) return "stretch needs omega_e > 0 and chi_e >= 0";
  const double quantum = (kPlanck * kLight) * we;
  const double anharm = quantum * xe;
  if (!(de > 0.0)) {
    if (!(xe > 0.0)) return "D_e missing and chi_e = 0";
    de = quantum / (4.0 * xe);
  }
  for (uint32_t i = 0; i < kLadderMax; ++i) {
    const double v = (double)i + 0.5;
    const double e = (quantum * v) - ((anharm * v) * v);
    if (!(e < de)) break;                         // dissociation limit
    if (!levels.empty() && !(e > levels.back())) break;  // past the turning point of the parabola
    levels.push_back(e);
  }
  return levels.empty() ? "stretch has no bound level" : nullptr;
}

const char *explicit_ladder(const double *e, uint32_t n, double de, std::vector<double> &levels) {
  levels.clear();
  if (!(de > 0.0)) return "explicit level list needs D_e > 0";
  for (uint32_t i = 0; i < n && i < kLadderMax && e[i] < de; ++i) {
    if (!levels.empty() && !(e[i] > levels.back())) return "level list must increase strictly";
    levels.push_back(e[i]);
  }
  return levels.empty() ? "stretch has no bound level" : nullptr;
}

// Series below x = a + 1 and a continued fraction (modified Lentz) above, the
// evaluation of Press et al., Numerical Recipes, sec. 6.2, stopping at a
// relative term of 1e-17 or after 1000 terms.
double upper_gamma_regularized(double a, double x) {
  if (!(x > 0.0)) return 1.0;
  const double log_front = -x + a * std::log(x) - std::lgamma(a);
  if (x < a + 1.0) {
    double denom = a, term = 1.0 / a, lower = term;
    for (int k = 0; k < 1000; ++k) {
      denom += 1.0;
      term *= x / denom;
      lower += term;
      if (std::fabs(term) < std::fabs(lower) * 1e-17) break;
    }
    return 1.0 - lower * std::exp(log_front);
  }
  const double floor_value = 1e-300;
  double b = (x + 1.0) - a;
  double cc = 1.0 / floor_value, dd = 1.0 / b, frac = dd;
  for (int k = 1; k <= 1000; ++k) {
    const double ak = -(double)k * ((double)k - a);
    b += 2.0;
    dd = ak * dd + b;
    if (std::fabs(dd) < floor_value) dd = floor_value;
    cc = b + ak / cc;
    if (std::fabs(cc) < floor_value) cc = floor_value;
    dd = 1.0 / dd;
    const double step = dd * cc;
    frac *= step;
    if (std::fabs(step - 1.0) < 1e-17) break;
  }
  return std::exp(log_front) * frac;
}

// bends as infinite harmonic ladders (1 / (1 - e^(-Theta/T)) each), stretches
// summed over their bound levels; modes multiplied in mode order
double partition_function(const ModeSet &m, double t) {
  double q = 1.0;
  for (double th : m.theta) q *= 1.0 / (1.0 - std::exp(-th / t));
  for (const std::vector<double> *L : m.ladder) {
    double z = 0.0;
    for (double level : *L) z += std::exp(-(level - (*L)[0]) / (kBoltzmann * t));
    q *= z;
  }
  return q;
}

double mean_energy(const ModeSet &m, double t) {
  double e = 0.0;
  for (double th : m.theta) e += kBoltzmann * th / std::expm1(th / t);
  for (const std::vector<double> *L : m.ladder) e += ladder_mean(*L, kBoltzmann * t, false);
  return e;
}

// bisection in log T on [1 K, 1e6 K] (the mean energy grows with T)
double vibrational_temperature(const ModeSet &m, double e) {
  if (m.size() == 0 || !(e > 0.0)) return 0.0;
  double lo = 0.0, hi = std::log(1.0e6);
  if (mean_energy(m, std::exp(hi)) < e) return std::exp(hi);
  for (int it = 0; it < 200 && hi - lo > 1e-15; ++it) {
    const double mid = 0.5 * (lo + hi);
    (mean_energy(m, std::exp(mid)) < e ? lo : hi) = mid;
  }
  return std::exp(0.5 * (lo + hi));
}

VibrationalThermometer::VibrationalThermometer(const ModeSet &m) : theta_(m.theta) {
  for (const std::vector<double> *L : m.ladder) ladders_.push_back(*L);
  constexpr int kGrid = 512;
  const double top = std::log(1.0e6);
  for (int i = 0; i < kGrid; ++i) {
    const double lt = top * (double)i / (double)(kGrid - 1);
    log_t_.push_back(lt);
    mean_.push_back(mean(std::exp(lt)));
  }
}

double VibrationalThermometer::mean(double t) const {
  double e = 0.0;
  for (double th : theta_) e += kBoltzmann * th / std::expm1(th / t);
  for (const std::vector<double> &L : ladders_) e += ladder_mean(L, kBoltzmann * t, false);
  return e;
}

double VibrationalThermometer::temperature(double e) const {
  if (theta_.empty() && ladders_.empty()) return 0.0;
  if (!(e > 0.0)) return 0.0;
  if (!(e < mean_.back())) return std::exp(log_t_.back());
  // first grid node whose mean energy reaches e
  size_t hi = (size_t)(std::lower_bound(mean_.begin(), mean_.end(), e) - mean_.begin());
  if (hi == 0) hi = 1;
  double a = log_t_[hi - 1], b = log_t_[hi];
  double fa = mean_[hi - 1] - e, fb = mean_[hi] - e;
  if (fb == 0.0) return std::exp(b);
  int side = 0;
  for (int it = 0; it < 100 && b - a > 1e-15 * (1.0 + std::fabs(b)); ++it) {
    const double x = (a * fb - b * fa) / (fb - fa);
    const double fx = mean(std::exp(x)) - e;
    if (fx == 0.0) return std::exp(x);
    if ((fx < 0.0) == (fa < 0.0)) {
      a = x;
      fa = fx;
      if (side == -1) fb *= 0.5;
      side = -1;
    } else {
      b = x;
      fb = fx;
      if (side == 1) fa *= 0.5;
      side = 1;
    }
    if (x == a && x == b) break;
  }
  return std::exp(std::fabs(fa) < std::fabs(fb) ? a : b);
}

double wr_probability(const ModeSet &m, double de, double omega, uint32_t n_samp, double t) {
  // oscillator frequencies: bends k Theta / h, stretches (E_1 - E_0) / h
  std::vector<double> nu;
  for (double th : m.theta) nu.push_back((kBoltzmann * th) / kPlanck);
  for (const std::vector<double> *L : m.ladder) nu.push_back(((*L)[1] - (*L)[0]) / kPlanck);
  double s1 = 0.0, s2 = 0.0;
  for (double f : nu) {
    s1 = s1 + f;
    s2 = s2 + f * f;
  }
  const double l = (double)nu.size();
  const double ez = 0.5 * kPlanck * s1;                  // zero-point energy E_z
  const double beta_wr = ((l - 1.0) * (l - 1.0) * s2) / (l * (s1 * s1));
  const double a_gamma = 2.5 - omega;
  double weighted = 0.0, total = 0.0;
  for (uint32_t k = 0; k < n_samp; ++k) {
    const double e = (double)k * de / (double)(n_samp - 1);
    const double r = e / ez;
    // Whitten-Rabinovich correction: two branches meeting at E = E_z
    const double w_corr = r >= 1.0 ? std::pow(10.0, -1.0506 * std::pow(r, 0.25))
                                   : 1.0 / (5.0 * r + 2.73 * std::sqrt(r) + 3.51);
    const double rho = std::pow(e + (1.0 - beta_wr * w_corr) * ez, l - 1.0);
    const double w = rho * std::exp(-e / (kBoltzmann * t));
    weighted += upper_gamma_regularized(a_gamma, (de - e) / (kBoltzmann * t)) * w;
    total += w;
  }
  return total > 0.0 ? weighted / total : 0.0;
}

double recombination_node(double l0, double inv_step, uint32_t i) { return std::exp(l0 + (double)i / inv_step); }

// ((((2 pi k T) / h^2)^(3/2) (m_B m_C / m_A)^(3/2)) (Q_B Q_C / Q_A)) exp(-dE0 / kT),
// dE0 = ((h_B + ZPE_B) + (h_C + ZPE_C)) - (h_A + ZPE_A)
double equilibrium_constant(const Recombination &r, double t) {
  const double ground = ((r.formation_b + r.zpe_b) + (r.formation_c + r.zpe_c)) - (r.formation_a + r.zpe_a);
  const double thermal = (2.0 * kPiHost * kBoltzmann * t) / (kPlanck * kPlanck);
  const double vib = (partition_function(*r.b, t) * partition_function(*r.c, t)) / partition_function(*r.a, t);
  return std::pow(thermal, 1.5) * std::pow((r.mass_b * r.mass_c) / r.mass_a, 1.5) * vib *
         std::exp(-ground / (kBoltzmann * t));
}

void recombination_factors(const Recombination &r, double l0, double inv_step, uint32_t n_nodes,
                           std::vector<double> &out) {
  const size_t n_third = r.m_mass.size();
  const size_t base = out.size();
  out.resize(base + n_third * n_nodes, 0.0);
  const double bc_omega = 1.0 - r.bc_esg;
  for (uint32_t i = 0; i < n_nodes; ++i) {
    const double t = recombination_node(l0, inv_step, i);
    const double keq = equilibrium_constant(r, t);
    const double rate_bc = maxwell_sigma_g(r.bc_dref, bc_omega, r.bc_tref, r.bc_mr, t);
    // forward probabilities per (A, M) exponent at this node
    std::vector<std::pair<double, double>> prob;
    for (size_t m = 0; m < n_third; ++m) {
      const double w = (r.omega_a + r.m_omega[m]) * 0.5;
      const double d = (r.dref_a + r.m_dref[m]) * 0.5;
      const double tr = (r.tref_a + r.m_tref[m]) * 0.5;
      double p = -1.0;
      for (const auto &pw : prob)
        if (pw.first == w) p = pw.second;
      if (p < 0.0 && r.exact)
        for (const auto &ex : *r.exact)
          if (ex.first == w) p = ex.second[i];
      if (p < 0.0) p = wr_probability(*r.a, r.de, w, r.n_samp, t);
      prob.emplace_back(w, p);
      const double mu = (r.mass_a * r.m_mass[m]) / (r.mass_a + r.m_mass[m]);
      const double symmetry = m == r.self ? 2.0 : 1.0;  // identical collision partners
      // k_f = P ((2 d^2) / symmetry) sqrt(((2 pi) k tr) / mu) (t / tr)^(1 - w)
      const double kf = p * ((2.0 * (d * d)) / symmetry) * std::sqrt((2.0 * kPiHost * kBoltzmann * tr) / mu) *
                        std::pow(t / tr, 1.0 - w);
      const double v = (kf / keq) / rate_bc;
      out[base + m * n_nodes + i] = std::isnan(v) || v < 0.0 ? 0.0 : v;
    }
  }
}

double exact_beta_grid(uint32_t j) { return std::ldexp(1.0 + (double)(j & 15u) / 16.0, (int)(j >> 4) + 40); }

void exact_beta_bins(const std::vector<double> &bend_kt, const ModeSet &m, double q, uint32_t lo_bin,
                     uint32_t hi_bin, uint32_t n_grid, std::vector<double> &out) {
  // mean proposal energy G(beta): bends k Theta / expm1(beta k Theta), stretches
  // their Boltzmann means at beta, modes in order
  auto g_of = [&](double beta) {
    double g = 0.0;
    for (double kt : bend_kt) g += kt / std::expm1(beta * kt);
    for (const std::vector<double> *L : m.ladder) g += ladder_mean(*L, beta, true);
    return g;
  };
  for (uint32_t bin = lo_bin; bin <= hi_bin; ++bin) {
    // the bin's midpoint energy: exponent and top mantissa bits from the bin,
    // then the next bit set
    const uint64_t bits = ((uint64_t)bin << 48) | (1ull << 47);
    double e_mid;
    std::memcpy(&e_mid, &bits, sizeof(e_mid));
    // smallest grid index whose G(beta) + q / beta is at most E'
    uint32_t first = 0, last = n_grid - 1;
    while (first != last) {
      const uint32_t probe = (first + last) >> 1;
      const double beta = exact_beta_grid(probe);
      if (g_of(beta) + q / beta <= e_mid)
        last = probe;
      else
        first = probe + 1;
    }
    out.push_back(exact_beta_grid(first));
  }
}

}  // namespace host
}  // namespace hcao
