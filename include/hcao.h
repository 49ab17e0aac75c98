/*
 * hcao.h -- C ABI of the MI355X (gfx950) HCAO DSMC collision-step library.
 *
 * The library advances independent 0D reservoir cells of a dilute gas by
 * the Direct Simulation Monte Carlo collision step with the polyatomic
 * harmonically-coupled-anharmonic-oscillator (HCAO) vibrational model of
 * Lauterbach, Tuttas and Pfeiffer, "A harmonically-coupled-anharmonic-
 * oscillator approach for polyatomic chemistry modeling in DSMC":
 *   - stretches are Morse oscillators (Eq. energy-AHO, chi_e = hc w_e/(4 D_e)),
 *     bends are harmonic (Eq. energy-SHO and its Theta form), local-mode basis
 *     (Sec. "The polyatomic HCAO model");
 *   - every accepted pair first tests the reaction channels (Sec. "Polyatomic
 *     QK reaction modeling": dissociation per stretch, Eq. Ecoll-diss;
 *     exchange with steric factor and mode coupling alpha_j, Eq. Ecoll-exch;
 *     competing channels weighted by their excess energy), else relaxes its
 *     molecules by the joint Larsen-Borgnakke acceptance (Sec. "Implementation
 *     of the polyatomic HCAO model") and scatters isotropically (VHS).
 * Pair selection is Bird's no-time-counter (NTC) scheme over disjoint pairs
 * of a keyed permutation; random numbers are Philox4x32-10 streams keyed by
 * (seed, step, cell, pair), so results do not depend on launch shape.
 *
 * Conventions
 *   Units: SI. Energies in J, measured from the potential minimum (they
 *   include zero-point energy). Velocities in m/s.
 *   Ownership: every input array is owned by the caller and copied during
 *   the call; output arrays are caller-allocated with the sizes documented
 *   below. All pointers are HOST pointers unless a name ends in _dev.
 *   The context owns its device memory (freed by hcao_destroy).
 *   Errors: every call returns an hcao_status. A device-side error (capacity
 *   overflow, non-finite state) is sticky: later calls return it until
 *   hcao_destroy. hcao_last_error() describes the last failure. No C++
 *   exception crosses this boundary.
 *   Call order: create -> add_species* -> add_reaction* -> finalize ->
 *   (load_particles | init_thermal) -> (step | read_*)*. Violations return
 *   HCAO_ESTATE.
 *   Threading: a context is not thread-safe. All device work is issued on
 *   the HIP stream given at create time (NULL = the null stream).
 *   Layout of level arrays: n x max_modes row-major uint16 quantum numbers;
 *   modes are ordered bends first, then stretches, as registered; unused
 *   slots (mode >= the species' mode count) must be 0.
 */
#ifndef HCAO_H
#define HCAO_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HCAO_ABI_VERSION 1u
#define HCAO_MAX_SPECIES 16
#define HCAO_MAX_MODES 16
#define HCAO_MAX_REACTIONS 32
#define HCAO_MAX_LEVELS 1024
/* per-cell counters (hcao_read_cell_state): */
#define HCAO_CTR_CANDIDATES 0 /* NTC candidate pairs tested */
#define HCAO_CTR_COLLISIONS 1 /* accepted pairs, reactive ones included */
#define HCAO_CTR_TRIALS 2     /* relaxation sampler trials */
#define HCAO_CTR_RELAX 3      /* molecule relaxations */
#define HCAO_CTR_CAPPED 4     /* sampler stopped after 1e6 trials (levels kept) */
#define HCAO_CTR_SUPPRESSED 5 /* NTC candidates beyond floor(N/2) (dropped), and
                                 recombinations without third body or energy */
#define HCAO_CTR_BIRTHS 6
#define HCAO_CTR_DEATHS 7
#define HCAO_CTR_REACTION0 8  /* + reaction id: reactions performed */
#define HCAO_N_CTR (8 + HCAO_MAX_REACTIONS)

typedef struct hcao_ctx hcao_ctx;

typedef enum {
  HCAO_OK = 0,
  HCAO_EINVAL = -1,      /* bad argument */
  HCAO_ESTATE = -2,      /* call out of order */
  HCAO_ENOMEM = -3,      /* host or device allocation failed */
  HCAO_EDEVICE = -4,     /* HIP runtime error */
  HCAO_ECAPACITY = -5,   /* a cell exceeded its slot capacity (births) */
  HCAO_ELEVEL = -6,      /* quantum number above the top bound level, or a
                            nonzero level in an unused mode slot */
  HCAO_ENONFINITE = -7,  /* non-finite velocity */
  HCAO_EUNSUPPORTED = -8, /* feature not available in this mode of the library */
  HCAO_EBOUNDS = -9       /* bounds-checked build (libhcao_checked.so) only: a
                             kernel formed a particle-slot or per-pair record
                             index outside its array; the access was redirected
                             to index 0, so the call's results are void. Sticky. */
} hcao_status;

/* Arithmetic of the step.
 *   HCAO_FP64: everything in IEEE fp64; bit-identical across launch shapes
 *     and to the fp64 reference of the method.
 *   HCAO_MIXED: velocities are stored in fp32; the VHS acceptance (g^2 and
 *     the power), the Larsen-Borgnakke draws, ratio and power, the level
 *     proposals and the post-collision kinematics run in fp32; collision
 *     energies, energy pools, reaction thresholds, channel weights and all
 *     accumulators stay fp64. Random draws take one 32-bit word each. The
 *     energy each collision's fp32 velocities gain or lose is audited in
 *     fp64 per cell and returned to the cell's particles in a later
 *     collision (hcao_moments.E_defect_J holds what is still owed).
 *     Results are reproducible and independent of launch shape, but not
 *     bit-identical to HCAO_FP64. */
typedef enum { HCAO_FP64 = 0, HCAO_MIXED = 1 } hcao_precision;
typedef enum {
  HCAO_SAMPLER_AUTO = 0,
  HCAO_SAMPLER_JOINT = 1,
  HCAO_SAMPLER_GIBBS = 2,
  HCAO_SAMPLER_EXACT = 3
} hcao_sampler;
typedef enum { HCAO_RX_DISSOCIATION = 0, HCAO_RX_EXCHANGE = 1, HCAO_RX_RECOMBINATION = 2 } hcao_rx_kind;
/* Forward probability of a recombination: the Whitten-Rabinovich
 * approximation, or the sum over every level combination (Eq. recomb-correct,
 * evaluated on the device at finalize). */
typedef enum { HCAO_REC_WR = 0, HCAO_REC_EXACT = 1 } hcao_rec_model;

/* Context configuration.
 *   seed: key of every random stream.
 *   n_cells: number of independent reservoir cells (>= 1).
 *   cell_volume / cell_weight: per-cell V [m^3] and particle weight F_N
 *     (real molecules per simulated particle); both must be > 0.
 *   capacity_per_cell: slot capacity of every cell; 0 = N + N/4 + 32 for a
 *     cell loaded with N particles. Dissociation appends products; a cell
 *     that would exceed its capacity stops the run with HCAO_ECAPACITY.
 *   device: HIP device ordinal. hip_stream: hipStream_t or NULL. */
typedef struct {
  uint32_t abi_version; /* must be HCAO_ABI_VERSION */
  hcao_precision precision;
  uint64_t seed;
  uint32_t n_cells;
  const double *cell_volume; /* n_cells */
  const double *cell_weight; /* n_cells */
  uint32_t capacity_per_cell;
  int device;
  void *hip_stream;
} hcao_config;

/* One species (Sec. "Implementation of the polyatomic HCAO model": every
 * stretch needs its level list or spectroscopic constants, every bend its
 * characteristic temperature).
 *   mass_kg; VHS d_ref [m], omega (0.5 <= omega < 1.5), T_ref [K];
 *   n_bend, bend_theta_K[n_bend];
 *   n_stretch, omega_e_per_m[n_stretch] (w_e in m^-1), chi_e[n_stretch],
 *     De_J[n_stretch] (<= 0 or NULL: hc w_e / (4 chi_e));
 *   n_levels / levels_J: optional explicit stretch level lists (NULL = Morse
 *     from w_e, chi_e), concatenated per stretch, strictly increasing;
 *   levels are kept while below D_e and still increasing (at most 1024);
 *   formation_J: formation energy h_s (reaction enthalpies are differences);
 *   coupling: stored and reported only (the pooled joint redistribution is
 *     the stretch-bend coupling of this model);
 *   p_vib: probability that an accepted non-reactive collision relaxes the
 *     molecule (0..1);
 *   sampler: JOINT = the joint proposal + acceptance as printed; GIBBS = one
 *     sweep of single-mode conditionals of the same target; EXACT = an
 *     independent draw from the joint target (E_coll - sum E_m)^q like JOINT,
 *     by rejection from per-mode Boltzmann proposals at one inverse
 *     temperature, whose acceptance does not collapse with many modes
 *     (about 3 trials for 9 modes); AUTO = JOINT for 2 to 4 modes, GIBBS
 *     otherwise (for one mode both have the same target, and the sweep's
 *     proposal accepts more often);
 *   zeta_rot: rotational degrees of freedom (0: no rotor, 2: linear, 3:
 *     nonlinear); the rotational energy is continuous, relaxed in each
 *     non-reactive collision (after the vibrational relaxation) with
 *     probability p_rot by the Larsen-Borgnakke rule: the rotor keeps a
 *     share f of E_tr + E_rot with density f^(zeta/2-1) (1-f)^(3/2-omega);
 *     thermal initialization draws it from Gamma(zeta/2, k T_trans). */
typedef struct {
  double mass_kg, dref_m, omega, Tref_K;
  uint32_t n_bend;
  const double *bend_theta_K;
  uint32_t n_stretch;
  const double *omega_e_per_m, *chi_e, *De_J;
  const uint32_t *n_levels;
  const double *levels_J;
  double formation_J;
  double coupling;
  double p_vib;
  hcao_sampler sampler;
  uint32_t zeta_rot;
  double p_rot;
} hcao_species_desc;

/* One reaction (Sec. "Polyatomic QK reaction modeling").
 *   DISSOCIATION: reactant[0] = A (any partner M), product = {B, C}; B takes
 *     A's slot, C is appended to the cell. stretch_mask bit j: A's j-th
 *     stretch is a dissociation channel (threshold: Eq. Ecoll-diss > D_e).
 *     m_A must equal m_B + m_C.
 *   EXCHANGE: reactant = {A, B}, product = {C, D}; C takes A's slot, D B's.
 *     alpha[n_modes of A] couples each of A's modes (Eq. Ecoll-exch); steric
 *     in [0,1]; Ea_J the barrier. m_A + m_B must equal m_C + m_D.
 *   RECOMBINATION (Sec. "Recombination reactions"): reactant = {B, C}
 *     (distinct species), product[0] = A, stretch_mask names the bond of A
 *     whose D_e enters the forward probability; rec_model picks the forward
 *     probability P: HCAO_REC_WR (the Whitten-Rabinovich approximation with
 *     n_samp sample energies, 0 = 1000) or HCAO_REC_EXACT (Eq.
 *     recomb-correct summed over every level combination of A on the device,
 *     see hcao_recombination_exact). The pair k's third
 *     body is the particle at permutation index 2 N_cand + k (if any); the
 *     pair recombines with probability min(1, k_b n / <sigma g>_BC) at the
 *     cell's step-start translational temperature, k_b = k_f / K_eq with k_f
 *     of the section's forward-rate expression (VHS means of A and the third
 *     body) and K_eq from translational and vibrational partition sums. B
 *     takes A's slot; C is removed. m_A must equal m_B + m_C.
 *   gamma_rot (Sec. "Rotation coupling"): degree of coupling in [0, 1];
 *     dissociation and exchange add gamma E_rot,A to the collision energies
 *     of Eqs. Ecoll-diss and Ecoll-exch and to the reaction's energy pool;
 *     the rest of A's rotation stays with the product in A's slot, B's with
 *     the product in B's slot (a product without a rotor pools it). Must be
 *     0 for a recombination, which hands B's and C's rotation to A. */
typedef struct {
  hcao_rx_kind kind;
  int32_t reactant[2];
  int32_t product[2];
  uint64_t stretch_mask;
  const double *alpha;
  double steric, Ea_J;
  double gamma_rot;
  uint32_t n_samp;
  hcao_rec_model rec_model;
} hcao_reaction_desc;

/* Moments of one cell or of all cells (hcao_read_moments).
 * E_trans_J is the translational energy in the frame of the cell's mean
 * velocity; T_trans_K = 2 E_trans / (3 k N); T_vib_K[s] solves the Boltzmann
 * mean-energy equation of the paper for the species' mean vibrational
 * energy above the zero point (0 for atoms or absent species). */
typedef struct {
  uint64_t n_total;
  uint64_t n_species[HCAO_MAX_SPECIES];
  double number_density[HCAO_MAX_SPECIES]; /* N_s F_N / V [m^-3] (total: summed over cells / total V) */
  double momentum[3];                      /* sum m v [kg m/s] per simulated particle */
  double E_trans_J, E_kin_J;               /* translational energy (COM frame), kinetic energy */
  double E_vib_J[HCAO_MAX_SPECIES];        /* sum of vibrational energy above the zero point */
  double E_formation_J;                    /* sum of formation energies */
  double T_trans_K;
  double T_vib_K[HCAO_MAX_SPECIES];
  double E_defect_J; /* mixed form: energy owed to the particles by fp32 rounding, not yet
                        returned (0 in HCAO_FP64); E_kin + sum (E_vib + N_s ZPE_s + E_rot)
                        + E_formation + E_defect is conserved to fp64 rounding */
  double E_rot_J[HCAO_MAX_SPECIES]; /* sum of rotational energy */
  double T_rot_K[HCAO_MAX_SPECIES]; /* 2 E_rot / (zeta k N_s) (0 without a rotor) */
} hcao_moments;

/* Spatial mode (the steps either side of the collision step): the cells
 * tile the box [0, lx) x [0, ly) x [0, lz) as an nx x ny x nz grid, cell =
 * ix + nx (iy + ny iz); bit k of periodic makes axis k periodic, else its
 * two walls reflect specularly. */
typedef struct {
  uint32_t nx, ny, nz, periodic;
  double lx, ly, lz;
} hcao_domain;

/* Open faces of the spatial mode (surface-flux boundaries; the paper's
 * cases are 0D reservoirs). Face f = 2 axis + side lies on that axis at 0
 * (side 0) or at L (side 1); bit f of open_faces opens it. A particle whose
 * move crosses an open face leaves the box. Every step, after the move,
 * face cell j of an open face (numbered over all six faces in face order,
 * j = i_a + n_a i_b on the face's tangential axes a < b) admits, per species
 * s, floor(x) particles with x = ((F_s A) dt) / F_N + rem, F_s = n_s sqrt(k
 * T_trans / (2 pi m_s)) the one-sided flux of a resting Maxwellian
 * reservoir, A the face cell's area, F_N the weight of the cell behind it,
 * rem the fraction carried from the previous step. Admission i of species s
 * draws from the stream (pair (s << 24) | i, cell n_cells + j, the step):
 * normal speed sigma sqrt(-2 ln(1 - u)) inward (sigma^2 = k T_trans / m_s),
 * the two tangential components sigma times a polar normal pair, the
 * fraction tau of the step it flies, its place uniform on the face cell per
 * tangential axis, then levels at T_vib and rotational energy at T_trans as
 * hcao_init_thermal draws them; it enters at the face and moves over tau dt
 * (and may leave again). Within a cell, admitted particles follow the
 * particles already in the box, in the order they were made.
 * number_density[n_species] in m^-3 (caller-owned, copied). */
typedef struct {
  uint32_t open_faces, pad;
  const double *number_density;
  double t_trans_K, t_vib_K;
} hcao_inflow;

const char *hcao_status_string(hcao_status s);
const char *hcao_last_error(const hcao_ctx *ctx);

hcao_status hcao_create(const hcao_config *cfg, hcao_ctx **out);
hcao_status hcao_add_species(hcao_ctx *ctx, const hcao_species_desc *sp, int32_t *id);
hcao_status hcao_add_reaction(hcao_ctx *ctx, const hcao_reaction_desc *rx, int32_t *id);
/* Turns on the spatial mode (before finalize): particles carry positions
 * [m]; every step moves each particle ballistically over dt (periodic axes
 * wrap into [0, L), the others reflect: x < 0 -> -x, x > L -> 2L - x, the
 * velocity component reversed, until inside), re-bins all particles by a
 * stable counting sort on their new cell on the device (within a cell the
 * previous cell-major order is kept), and then collides. n_cells must be
 * nx ny nz and every cell volume the grid cell's. A cell that would exceed
 * its slot capacity raises HCAO_ECAPACITY. hcao_step_graph and
 * hcao_autotune are not available in this mode (HCAO_EUNSUPPORTED). */
hcao_status hcao_set_domain(hcao_ctx *ctx, const hcao_domain *domain);
/* Opens faces of the spatial mode to a reservoir (after finalize; before
 * the particles are loaded or at any later point: the inflow remainders and
 * flux counts start at zero here and at every load, init and restore).
 * open_faces 0 closes them again. HCAO_ESTATE outside the spatial mode,
 * HCAO_EINVAL for an open face on a periodic axis, a negative or
 * non-finite density or a non-positive temperature. A checkpoint of a
 * context with open faces restores only into a context with open faces. */
hcao_status hcao_set_inflow(hcao_ctx *ctx, const hcao_inflow *inflow);
/* out[0]: particles admitted through open faces, out[1]: particles that
 * left through them (admissions that leave again during their first flight
 * included), since the last load, init or restore; zeros without open faces. */
hcao_status hcao_read_flux_counts(hcao_ctx *ctx, uint64_t out[2]);
/* Builds the level, pair and reaction tables and uploads them. */
hcao_status hcao_finalize(hcao_ctx *ctx);

/* Loads n particles from host arrays in any order: cell[n] (< n_cells),
 * species[n], vel[3n] (x,y,z per particle), levels[n * max_modes].
 * rot[n] (may be NULL: none) rotational energies [J], >= 0 and 0 for
 * species without a rotor; pos[3n] positions [m] (spatial mode: required,
 * inside the box and in the particle's cell; otherwise ignored). Particles
 * are placed by a stable counting sort
 * on the device, so each cell keeps the given relative order. Resets the
 * step counter to 0 and sets each cell's (sigma g)_max to an upper bound
 * over its initial pairs. */
hcao_status hcao_load_particles(hcao_ctx *ctx, uint64_t n, const uint32_t *cell, const uint8_t *species,
                                const double *vel, const uint16_t *levels, const double *rot, const double *pos);

/* Thermal initial state on the device: counts[n_cells * n_species] particles
 * per cell and species (species-major within a cell), Maxwellian velocities
 * at t_trans[c] and vibrational levels at t_vib[c] (the paper's
 * initialization: bends by the floor form, stretches by Eq. accept-quant
 * with a proposal over 0..i_diss), rotational energies of rotors from
 * Gamma(zeta/2, k t_trans[c]) and, in the spatial mode, positions uniform
 * in the cell. */
hcao_status hcao_init_thermal(hcao_ctx *ctx, const uint32_t *counts, const double *t_trans,
                              const double *t_vib);

/* Advances every cell by n_steps collision steps of length dt [s]. */
hcao_status hcao_step(hcao_ctx *ctx, double dt, uint32_t n_steps);

/* Launch shape of the step kernel. Results do not depend on it, bit for
 * bit: it only changes how cells map onto workgroups and launches.
 *   block: workgroup size, 64, 128, 256 or 512 lanes;
 *   group_slots: a workgroup takes consecutive cells while their summed slot
 *     capacity stays within group_slots (at least one cell, at most 64, and
 *     fewer when the workgroup's per-cell LDS records would not fit);
 *   steps_per_launch: steps one kernel launch advances, each workgroup
 *     keeping its cells' state in LDS between them (0 = all steps of a call).
 * Defaults 64, 1024, 0; the environment variables HCAO_BLOCK,
 * HCAO_GROUP_SLOTS and HCAO_STEPS_PER_LAUNCH override them at create time.
 * hcao_set_launch_shape waits for the stream; it returns HCAO_EINVAL for a
 * block size not listed or group_slots = 0. */
typedef struct {
  uint32_t block;
  uint32_t group_slots;
  uint32_t steps_per_launch;
} hcao_launch_shape;
hcao_status hcao_get_launch_shape(const hcao_ctx *ctx, hcao_launch_shape *shape);
hcao_status hcao_set_launch_shape(hcao_ctx *ctx, const hcao_launch_shape *shape);

/* Autotuner of the launch shape: times trial_steps steps of every candidate
 * (block 64, 128, 256 x group_slots 256 .. 6144) from a device copy of the
 * current state advanced by max(trial_steps, 10) steps (so that the first
 * steps' settling (sigma g)_max does not decide), puts the state back, and
 * keeps the fastest candidate. Trials shorter than one launch
 * (steps_per_launch) weigh a launch's start and tail more than the timed
 * configuration does and can prefer larger workgroups (on the 67 M-particle
 * chemistry: 5-step trials choose 4096 slots, 50-step trials 2048, the
 * faster one over 50-step launches)
 * (steps_per_launch is left as it is). The particles, per-cell state,
 * counters and step index after the call are those before it. cache_path
 * (or, when NULL, the environment variable HCAO_AUTOTUNE_CACHE; no cache if
 * neither is set) names a text file of earlier results keyed by cell
 * layout, species set and precision: a hit is used without timing, a new
 * result is appended. chosen may be NULL. Needs loaded particles. */
hcao_status hcao_autotune(hcao_ctx *ctx, double dt, uint32_t trial_steps, const char *cache_path,
                          hcao_launch_shape *chosen);

/* hipGraph form of hcao_step: the first call for a given (dt, n_steps) and
 * launch shape captures the step-kernel launches of n_steps steps and a
 * device-side update of the step index into a graph on the context's
 * stream; later calls replay it. Results are bitwise those of hcao_step. */
hcao_status hcao_step_graph(hcao_ctx *ctx, double dt, uint32_t n_steps);

/* Allocation-free step, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same n_steps steps as hcao_step, with bitwise the same
 * result, but the step's work lists, pair flags, pair energy defects and
 * products staging live in one fixed device array of
 * HCAO_STATIC_SCRATCH_BYTES that the library holds on each GPU it runs on
 * until the process ends, not in the context's buffers. The call allocates
 * and frees nothing. Its need is about 30 + 3 b_v + 2 max_modes bytes per
 * work entry (b_v = 8 fp64, 4 mixed; 8 more in the mixed form, 8 more with
 * rotors and 40 more with a recombination reaction; work entries = sum over cells of capacity / 2 + 1, e.g.
 * 725,000 for 4,096 cells of 256 particles at the default capacity, 52 MB
 * in fp64 for the methane species): a context that needs more
 * gets HCAO_ECAPACITY with the figure in hcao_last_error and nothing runs.
 * The spatial mode is refused (HCAO_EUNSUPPORTED): its re-bin needs buffers
 * as large as the state. Every call on a GPU uses that GPU's one array, whose
 * contents the next call overwrites (nothing in it needs to start at zero):
 * calls that overlap on one GPU, from two streams or threads, race, and the
 * caller must order them. Asynchronous on the context's stream, like
 * hcao_step. */
#define HCAO_STATIC_SCRATCH_BYTES (128u << 20)
hcao_status hcao_step_static(hcao_ctx *ctx, double dt, uint32_t n_steps);

/* Waits for the stream and returns the sticky device status. */
hcao_status hcao_sync(hcao_ctx *ctx);

/* Sizes: number of cells' live particles and the mode-slot count. */
hcao_status hcao_get_counts(hcao_ctx *ctx, uint64_t *per_cell /* n_cells or NULL */, uint64_t *total);
uint32_t hcao_max_modes(const hcao_ctx *ctx);
uint32_t hcao_step_index(const hcao_ctx *ctx);

/* Reads every live particle in canonical order (cell-major; within a cell:
 * survivors in their previous order, then products born in pair order).
 * species[total], vel[3 total], levels[total * max_modes]. */
hcao_status hcao_read_particles(hcao_ctx *ctx, uint8_t *species, double *vel, uint16_t *levels);
/* Rotational energies [J] of every live particle, rot[total], in the order
 * of hcao_read_particles (all 0 when no species has a rotor). */
hcao_status hcao_read_rotational_energy(hcao_ctx *ctx, double *rot);
/* Positions [m] of every live particle, pos[3 total], in the order of
 * hcao_read_particles (spatial mode only, else HCAO_ESTATE). */
hcao_status hcao_read_positions(hcao_ctx *ctx, double *pos);

/* The live particles of one cell in canonical order (for sampled checks of
 * large runs): writes min(count, max_n) particles into species[max_n],
 * vel[3 max_n], levels[max_n * max_modes] and the cell's count into *n_out.
 * HCAO_EINVAL for a cell index >= n_cells. */
hcao_status hcao_read_cell_particles(hcao_ctx *ctx, uint32_t cell, uint32_t max_n, uint8_t *species, double *vel,
                                     uint16_t *levels, uint32_t *n_out);

/* Per-cell state: sgmax[n_cells] ((sigma g)_max, m^3/s), rem[n_cells] (NTC
 * remainder), counters[n_cells * HCAO_N_CTR]. Any pointer may be NULL. */
hcao_status hcao_read_cell_state(hcao_ctx *ctx, double *sgmax, double *rem, uint64_t *counters);

/* Moments; per_cell[n_cells] may be NULL. */
hcao_status hcao_read_moments(hcao_ctx *ctx, hcao_moments *per_cell, hcao_moments *total);

/* Reaction counts summed over cells: counts[n_reactions]. */
hcao_status hcao_read_reaction_counts(hcao_ctx *ctx, uint64_t *counts);

/* Tables as built on the host (for table-equality checks):
 * hcao_get_levels: stretch levels (or the first max_n bend levels) of one
 * mode, returns the count written via *n_out. hcao_get_pair: m_r, m_r/2,
 * m_a + m_b, m_b/(m_a+m_b), m_a/(m_a+m_b), C (sigma g = C (g^2)^e), e, q. */
hcao_status hcao_get_levels(const hcao_ctx *ctx, uint32_t species, uint32_t mode, double *out, uint32_t max_n,
                            uint32_t *n_out);
hcao_status hcao_get_pair(const hcao_ctx *ctx, uint32_t a, uint32_t b, double *out8);
/* Recombination probability factors k_b(T) / <sigma g>_BC(T) [m^3] of one
 * recombination reaction: n_species x 1024 values (third-body species major,
 * temperature nodes log-spaced on [100, 5e4] K). */
hcao_status hcao_get_recombination_table(const hcao_ctx *ctx, uint32_t reaction, double *out, uint32_t max_n,
                                         uint32_t *n_out);
/* Inverse temperature [1/J] of the EXACT sampler's proposal for a molecule
 * of `species` relaxing in a collision with `partner` (the pair's LB
 * exponent q), at energy e_J > 0 above the molecule's zero point: the value
 * the step kernel reads from its per-(species, q) table for that energy's
 * bin, raised to q / e_J if below. HCAO_EINVAL if the species does not use
 * the EXACT sampler, has no modes, or e_J is not positive. Host-side table
 * read; no device work. */
hcao_status hcao_get_exact_beta(const hcao_ctx *ctx, uint32_t species, uint32_t partner, double e_J, double *beta);

/* Forward recombination probability of Sec. "Recombination reactions",
 * Eq. recomb-correct, for product species `species` with bond energy de_J
 * and VHS omega (a = 5/2 - omega, 0.5 <= omega < 1.5), at n_t temperatures
 * t_K[] (host, K) into p_out[] (host). P(T) = sum_i Q(a, (D_e - S_i)/kT)
 * exp(-S_i/kT) / sum_i exp(-S_i/kT) over every combination i of the
 * species' vibrational levels, S_i its energy above the ground level, Q the
 * regularized upper incomplete gamma (1 for arguments <= 0); bends are
 * infinite harmonic ladders, stretches run to their top bound level. The
 * device enumerates every combination below D_e (one record each) and the
 * points where the enumeration first crosses D_e (the combinations above it
 * have Q = 1 and are summed in closed form there), then sums the records
 * for each temperature in one workgroup. Sums are in a fixed order, so
 * results repeat bitwise; they match a serial sum to rounding (~1e-13
 * relative). elapsed_ms and n_records (may be NULL) receive the device
 * time and the number of records. Allocates device memory for the records
 * (16 bytes each); synchronous on the context's stream. HCAO_EUNSUPPORTED
 * if the species' stretch ladders exceed 8192 levels in total. */
hcao_status hcao_recombination_exact(hcao_ctx *ctx, uint32_t species, double de_J, double omega, uint32_t n_t,
                                     const double *t_K, double *p_out, double *elapsed_ms, uint64_t *n_records);

/* Kernel timing over the stream: when enabled, each hcao_step call records
 * HIP events on the context's stream around its step-kernel launches;
 * hcao_kernel_time returns the summed elapsed milliseconds, the number of
 * launches and the number of steps they advanced since enabling (a launch
 * advances every cell by up to the shape's steps_per_launch steps; a graph
 * replay counts its step-kernel launches). */
hcao_status hcao_set_timing(hcao_ctx *ctx, int enable);
hcao_status hcao_kernel_time(hcao_ctx *ctx, double *ms, uint64_t *launches, uint64_t *steps);

/* Phase clocks of the step kernel, a debugging aid of instrumented builds
 * (library compiled with HCAO_PHASE_CLOCKS; the default build returns
 * HCAO_EUNSUPPORTED). Thread 0 of every step workgroup sums the shader
 * clock cycles (clock64) spent in each phase of the step; out[0..n) (n <=
 * HCAO_N_PHASES, host array) receives the sums over all workgroups since the
 * last reset, in the order: launch loads, NTC counts and permutation keys,
 * cell temperature, candidate acceptance, work-list sort, collisions,
 * product placement, launch stores; then the collision phase per wave
 * (summed over waves): gathering a pair's state, reaction decision,
 * relaxation sampler, scattering and reaction application, write-back.
 * The first call allocates the sums
 * (zero); reset != 0 zeroes them after reading. Synchronous on the
 * context's stream. */
#define HCAO_N_PHASES 13
hcao_status hcao_phase_clocks(hcao_ctx *ctx, uint64_t *out, uint32_t n, int reset);

/* Checkpoint of the full state (particles, per-cell state, step index). */
hcao_status hcao_save(hcao_ctx *ctx, const char *path);
hcao_status hcao_restore(hcao_ctx *ctx, const char *path);

void hcao_destroy(hcao_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif
