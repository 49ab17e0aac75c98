/*
 * hcao_oracle.h -- fp64 CPU oracle of the HCAO DSMC collision step.
 *
 * TEST INFRASTRUCTURE. This library exists only to check the GPU library
 * against a plain, slow, obviously correct implementation. Only the test
 * suite, the smoke entry point and the CPU-baseline leg of the benchmark
 * may load it. The product path never calls it, and it shares no source
 * with the GPU library: both are written independently from the paper
 * (Lauterbach, Tuttas, Pfeiffer, "A harmonically-coupled-anharmonic-
 * oscillator approach for polyatomic chemistry modeling in DSMC") and from a
 * shared determinism specification (counter-based streams, draw order,
 * deterministic log/exp) that fixes every random draw and rounding.
 *
 * Plain C API (ctypes friendly). Energies in J, SI units throughout.
 * Every call returns 0 on success and a negative code on error.
 */
#ifndef HCAO_ORACLE_H
#define HCAO_ORACLE_H
#include <stdint.h>

#define ORC_MAX_SPECIES 16
#define ORC_MAX_MODES 16
#define ORC_MAX_LEVELS 1024
#define ORC_MAX_REACTIONS 32
#define ORC_MAX_TRIALS 1000000

/* per-cell counter slots */
enum {
  ORC_CTR_CANDIDATES = 0, /* NTC candidate pairs tested */
  ORC_CTR_COLLISIONS = 1, /* accepted pairs (reactive ones included) */
  ORC_CTR_TRIALS = 2,     /* relaxation sampler trials */
  ORC_CTR_RELAX = 3,      /* relaxations performed */
  ORC_CTR_CAPPED = 4,     /* sampler gave up after ORC_MAX_TRIALS */
  ORC_CTR_SUPPRESSED = 5, /* NTC excess over floor(N/2); recombinations without third body or energy */
  ORC_CTR_BIRTHS = 6,
  ORC_CTR_DEATHS = 7,
  ORC_CTR_REACTION0 = 8,  /* + reaction id */
  ORC_N_CTR = 8 + ORC_MAX_REACTIONS
};

enum { ORC_SAMPLER_AUTO = 0, ORC_SAMPLER_JOINT = 1, ORC_SAMPLER_GIBBS = 2, ORC_SAMPLER_EXACT = 3 };
enum { ORC_RX_DISSOCIATION = 0, ORC_RX_EXCHANGE = 1, ORC_RX_RECOMBINATION = 2 };

typedef struct orc_ctx orc_ctx;

/* ---- determinism primitives (exported for pins) ---- */
void orc_philox4x32_10(uint32_t k0, uint32_t k1, const uint32_t ctr[4], uint32_t out[4]);
double orc_detlog(double x);
double orc_detexp(double x);
double orc_detpow(double x, double y);
uint32_t orc_feistel_index(uint32_t n, const uint32_t keys[16], uint32_t i);
/* Gibbs-sweep level proposal: weights 1 - c i on 0..top, by inversion of u */
uint32_t orc_gibbs_propose(uint32_t top, double c, double u);
/* inverse temperature of the exact sampler's proposal for a molecule of the
 * given species with LB exponent q and energy E' above its zero point
 * (-1 on invalid input) */
double orc_exact_beta(orc_ctx *o, uint32_t species, double q, double ep);

/* ---- context ---- */
int orc_create(uint64_t seed, uint32_t n_cells, const double *cell_volume, const double *cell_weight,
               uint32_t capacity_per_cell, orc_ctx **out);
void orc_destroy(orc_ctx *o);
int orc_add_species(orc_ctx *o, double mass, double dref, double omega, double tref,
                    uint32_t n_bend, const double *theta, uint32_t n_stretch, const double *omega_e,
                    const double *chi_e, const double *de, const uint32_t *n_levels,
                    const double *levels, double formation, double p_vib, int sampler);
int orc_add_reaction(orc_ctx *o, int kind, const int32_t reactant[2], const int32_t product[2],
                     uint64_t stretch_mask, const double *alpha, double steric, double ea, uint32_t n_samp);
/* rotational mode of a species: zeta in {0, 2, 3}, relaxation probability p_rot */
int orc_set_rotation(orc_ctx *o, uint32_t species, uint32_t zeta, double p_rot);
/* rotation coupling gamma in [0, 1] of a dissociation or exchange */
int orc_set_gamma_rot(orc_ctx *o, uint32_t reaction, double gamma);
int orc_finalize(orc_ctx *o);
/* rot[n] (may be NULL: all zero) holds rotational energies [J]; pos[3n]
 * positions (spatial mode, required there; else ignored) */
int orc_load(orc_ctx *o, uint64_t n, const uint32_t *cell, const uint8_t *species, const double *vel,
             const uint16_t *levels, const double *rot, const double *pos);
/* spatial mode: box of nx x ny x nz cells, periodic axes as bits 0..2 */
int orc_set_domain(orc_ctx *o, uint32_t nx, uint32_t ny, uint32_t nz, double lx, double ly, double lz,
                   uint32_t periodic);
int orc_read_pos(const orc_ctx *o, uint32_t cell, double *pos);
/* spatial mode, after finalize: faces f = 2 axis + side (side 1 at L) open
 * as bits of open, admitting from a resting reservoir of number densities
 * n_s[n_species] [m^-3] at t_trans and t_vib */
int orc_set_inflow(orc_ctx *o, uint32_t open, const double *n_s, double t_trans, double t_vib);
/* out[0] particles admitted, out[1] particles that left, since the last load */
int orc_flux_counts(const orc_ctx *o, uint64_t *out);
int orc_init_thermal(orc_ctx *o, const uint32_t *counts, const double *t_trans, const double *t_vib);
int orc_step(orc_ctx *o, double dt, uint32_t n_steps);
/* threads over cells for orc_step (cells are independent: same result) */
int orc_set_threads(orc_ctx *o, int n);

/* ---- queries ---- */
uint32_t orc_max_modes(const orc_ctx *o);
uint64_t orc_count(const orc_ctx *o, uint32_t cell);
uint32_t orc_step_index(const orc_ctx *o);
int orc_read_cell(const orc_ctx *o, uint32_t cell, uint8_t *species, double *vel, uint16_t *levels);
int orc_read_rot(const orc_ctx *o, uint32_t cell, double *rot);
int orc_rot_energy(const orc_ctx *o, uint32_t cell, double *per_species);
int orc_collide_rot_batch(orc_ctx *o, uint32_t n, const uint8_t *sp, const double *vel, const uint16_t *lvl,
                          const double *rot, uint8_t *sp_out, double *vel_out, uint16_t *lvl_out, double *rot_out,
                          int32_t *reaction_out, uint8_t *born_sp, double *born_vel, uint16_t *born_lvl,
                          double *born_rot);
int orc_read_cell_state(const orc_ctx *o, uint32_t cell, double *sgmax, double *rem, uint64_t *ctr);
int orc_levels(const orc_ctx *o, uint32_t species, uint32_t mode, double *out, uint32_t max_n);
int orc_species_info(const orc_ctx *o, uint32_t species, double *zpe, uint32_t *n_modes,
                     uint32_t *sampler);
int orc_pair_info(const orc_ctx *o, uint32_t a, uint32_t b, double *out8);
int orc_moments(const orc_ctx *o, uint32_t cell, double *out);
int orc_tvib(const orc_ctx *o, uint32_t species, double mean_evib_above_ground, double *t_out);

/* ---- single-operation drivers for statistical and brute-force pins ---- */
int orc_relax_batch(orc_ctx *o, uint32_t species, double q, int sampler, uint32_t n,
                    const double *e_tr, const uint16_t *lvl_in, uint16_t *lvl_out,
                    double *e_tr_out, uint64_t *trials);
int orc_relax_chain(orc_ctx *o, uint32_t species, double q, int sampler, uint32_t chain,
                    uint32_t n_iter, const double *e_tr, uint16_t *lvl_state, uint64_t *hist,
                    uint32_t hist_stride);
int orc_collide_batch(orc_ctx *o, uint32_t n, const uint8_t *sp, const double *vel,
                      const uint16_t *lvl, uint8_t *sp_out, double *vel_out, uint16_t *lvl_out,
                      int32_t *reaction_out, uint8_t *born_sp, double *born_vel, uint16_t *born_lvl);
/* ---- recombination (Sec. "Recombination reactions") ---- */
double orc_gamma_q(double a, double x);
double orc_wr_rho(const orc_ctx *o, uint32_t species, double e);
double orc_wr_probability(const orc_ctx *o, uint32_t species, double de, double omega, uint32_t n_samp, double t);
double orc_q_vib(const orc_ctx *o, uint32_t species, double t);
/* Eq. recomb-correct: the forward probability summed over every level
 * combination of the species (a = 5/2 - omega), at temperature t. */
double orc_rec_exact_probability(const orc_ctx *o, uint32_t species, double de, double omega, double t);
double orc_rec_factor(const orc_ctx *o, uint32_t reaction, uint32_t third, double t);
/* pieces of the recombination factor k_f / K_eq / <sigma g>_BC of a
 * recombination reaction (B + C + M -> A + M) at temperature t: the
 * equilibrium constant of A <-> B + C [m^-3], the forward rate coefficient
 * of A + M -> B + C + M [m^3/s] and its forward probability P; the
 * temperature of table node i */
double orc_equilibrium_constant(const orc_ctx *o, uint32_t reaction, double t);
double orc_forward_rate(const orc_ctx *o, uint32_t reaction, uint32_t third, double t);
double orc_forward_probability(const orc_ctx *o, uint32_t reaction, uint32_t third, double t);
double orc_rec_node_temperature(const orc_ctx *o, uint32_t i);
/* translational temperature of a cell as the next step takes it (from the
 * cell's running sums); the sums themselves (m, m v_x, m v_y, m v_z,
 * m |v|^2): running (direct = 0) or summed afresh over the particles
 * (direct = 1) */
double orc_cell_temperature(const orc_ctx *o, uint32_t cell);
int orc_cell_sums(const orc_ctx *o, uint32_t cell, int direct, double *out5);
/* draw i of n from the stream (seed; pair i, cell 0, step 0): scattering
 * unit vectors (out[3 n]) and the three-body energy share (out[n]) */
void orc_draw_unit_vectors(uint64_t seed, uint32_t n, double *out);
void orc_draw_three_body_shares(uint64_t seed, uint32_t n, double *out);
int orc_rec_table(const orc_ctx *o, uint32_t reaction, double *out);
int orc_collide3_batch(orc_ctx *o, uint32_t n, const uint8_t *sp, const double *vel, const uint16_t *lvl,
                       uint8_t *sp_out, double *vel_out, uint16_t *lvl_out, int32_t *reaction_out,
                       uint8_t *born_sp, double *born_vel, uint16_t *born_lvl, const uint8_t *m_sp, double *m_vel,
                       double t_cell, double n_cell);
#endif
