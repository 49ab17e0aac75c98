// hcao_host_tables.h -- host-side tables of the step: Morse level ladders,
// vibrational partition functions and mean energies, the recombination
// factors (forward probability, equilibrium constant, collision rates) and
// the exact sampler's inverse-temperature bins.
//
// Every value that feeds the device tables is evaluated in the expression
// order the determinism specification fixes (left to right as written in
// each function's comment, no contraction), so that an independent
// implementation of the same specification produces the same bits.
#pragma once
#include <stdint.h>

#include <vector>

namespace hcao {
namespace host {

// The vibrational modes of one species in mode order: bends first (by
// Theta), then stretches (by their level ladders, energies in J from the
// potential minimum).
struct ModeSet {
  std::vector<double> theta;                       // bends: Theta [K]
  std::vector<const std::vector<double> *> ladder;  // stretches: E_0 < E_1 < ... [J]
  uint32_t size() const { return (uint32_t)(theta.size() + ladder.size()); }
};

// Morse ladder (Eq. energy-AHO) of harmonic wavenumber w_e [1/m] and
// anharmonicity x_e: with a = (h c) w_e and v = i + 1/2, E_i = (a v) -
// ((a x_e) v) v, kept while below D_e and still increasing. de <= 0 means
// "not given": D_e = a / (4 x_e) (x_e > 0). Returns null on success, else
// the reason.
const char *morse_ladder(double we, double xe, double &de, std::vector<double> &levels);
// An explicit ladder: energies below D_e (> 0), strictly increasing.
const char *explicit_ladder(const double *e, uint32_t n, double de, std::vector<double> &levels);

// Regularized upper incomplete gamma Q(a, x), 1 for x <= 0.
double upper_gamma_regularized(double a, double x);

// Vibrational partition function from the ground level at temperature t.
double partition_function(const ModeSet &m, double t);
// Mean vibrational energy above the ground level at temperature t, and its
// inverse (the vibrational temperature of a mean energy; 0 for no modes).
double mean_energy(const ModeSet &m, double t);
double vibrational_temperature(const ModeSet &m, double e);

// The same inverse for many energies of one species: the mean energy on a
// log-spaced temperature grid over [1 K, 1e6 K] brackets the root, then a
// bracketed secant (Illinois) iteration on the exact mean energy in log T
// refines it to rounding. Holds its own copy of the modes.
class VibrationalThermometer {
 public:
  VibrationalThermometer() = default;
  explicit VibrationalThermometer(const ModeSet &m);
  double temperature(double e) const;

 private:
  double mean(double t) const;  // mean_energy over the copied modes
  std::vector<double> theta_;
  std::vector<std::vector<double>> ladders_;
  std::vector<double> log_t_, mean_;
};

// Whitten-Rabinovich forward probability of the recombination section at
// temperature t: D_e the bond energy, omega the (A, third body) VHS exponent,
// n_samp energies on [0, D_e].
double wr_probability(const ModeSet &m, double de, double omega, uint32_t n_samp, double t);

// Temperature of recombination table node i (log-spaced on [T_min, T_max]).
double recombination_node(double l0, double inv_step, uint32_t i);

// Inputs of one recombination reaction B + C (+M) -> A (+M).
struct Recombination {
  const ModeSet *a, *b, *c;
  double mass_a, mass_b, mass_c;          // [kg]
  double formation_a, formation_b, formation_c, zpe_a, zpe_b, zpe_c;  // [J]
  double dref_a, omega_a, tref_a;         // A's VHS data
  double bc_dref, bc_tref, bc_esg, bc_mr;  // B-C pair: mean d, mean T_ref, 1 - omega, reduced mass
  double de;                              // bond energy D_e [J]
  uint32_t n_samp;
  uint32_t self;                          // species index of A (identical-partner symmetry)
  // third bodies, by species index: VHS data and mass
  std::vector<double> m_dref, m_omega, m_tref, m_mass;
  // optional forward probabilities per node for an (A, M) exponent, used
  // instead of the WR probability (Eq. recomb-correct on the device)
  const std::vector<std::pair<double, std::vector<double>>> *exact;
};

// k_f / K_eq / <sigma g>_BC per third-body species (rows of n_nodes) on the
// node temperatures, appended to out.
void recombination_factors(const Recombination &r, double l0, double inv_step, uint32_t n_nodes,
                           std::vector<double> &out);
// K_eq(T) of A <-> B + C [m^-3].
double equilibrium_constant(const Recombination &r, double t);

// Exact sampler: beta per bin of E' for LB exponent q (bends by k Theta,
// stretches by their ladders), bins lo..hi, appended to out.
void exact_beta_bins(const std::vector<double> &bend_kt, const ModeSet &m, double q, uint32_t lo, uint32_t hi,
                     uint32_t n_grid, std::vector<double> &out);
double exact_beta_grid(uint32_t j);

}  // namespace host
}  // namespace hcao
