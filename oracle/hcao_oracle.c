/*
 * hcao_oracle.c -- fp64 CPU oracle of the HCAO DSMC collision step.
 *
 * TEST INFRASTRUCTURE ONLY (see hcao_oracle.h). Written for clarity, not
 * speed: one cell at a time, one pair at a time, in the order the method
 * states. Compile with -O2 -ffp-contract=off and without fast-math so that
 * every floating-point operation is the IEEE operation written here.
 *
 * Paper sections followed (Lauterbach, Tuttas, Pfeiffer):
 *   harmonic and Morse levels ....... Introduction, Eqs. energy-SHO, energy-AHO,
 *                                     chi_e = hc w_e / (4 D_e); Sec. "The polyatomic
 *                                     HCAO model" (theta form of the harmonic levels)
 *   vibrational temperature ......... Sec. "Implementation ...", mean-energy equation
 *   initial quantum numbers ......... same section, bend floor form and the stretch
 *                                     acceptance Eq. accept-quant
 *   relaxation ...................... same section: E_coll, bend/stretch i_max,
 *                                     joint Larsen-Borgnakke acceptance, xi_rel = 5 - 2w
 *   dissociation .................... Sec. "Dissociation reactions", Eq. Ecoll-diss
 *   exchange ........................ Sec. "Exchange reactions", Eq. Ecoll-exch
 *   competing reactions ............. Sec. "Competing reactions"
 *   product redistribution .......... Sec. "Polyatomic QK reaction modeling" (LB)
 *   rotation coupling ............... Sec. "Rotation coupling" (gamma E_rot in both
 *                                     collision energies; the rotor model is our own)
 *   exact recombination sum ......... Sec. "Recombination reactions", Eq. recomb-correct
 *   spatial mode .................... not in the paper (move, re-bin, collide)
 *   open faces ...................... not in the paper (outflow, admission from a
 *                                     resting Maxwellian reservoir; the admitted
 *                                     molecules' levels by the initial-state sampler)
 * Pieces the paper takes from elsewhere are written from their textbook
 * definitions: NTC candidate count and VHS cross-section (Bird), Marsaglia's
 * (1972) unit vector and polar normal method, Philox4x32-10 (Salmon et al.,
 * SC'11), Cody-Waite argument reduction (Cody & Waite 1980), a Feistel
 * network permutation (Luby & Rackoff 1988) with cycle walking (Black &
 * Rogaway 2002).
 */
#include "hcao_oracle.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

/* exact SI constants */
#define H_PLANCK 6.62607015e-34
#define C_LIGHT 299792458.0
#define K_BOLTZ 1.380649e-23
#define PI_D 3.141592653589793

enum { E_OK = 0, E_INVAL = -1, E_STATE = -2, E_NOMEM = -3, E_CAPACITY = -5, E_LEVEL = -6, E_NONFINITE = -7 };

/* ------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11)                   */
/* ------------------------------------------------------------------ */
void orc_philox4x32_10(uint32_t k0, uint32_t k1, const uint32_t ctr[4], uint32_t out[4]) {
  uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    uint64_t prod0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
    uint64_t prod1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
    uint32_t hi0 = (uint32_t)(prod0 >> 32), lo0 = (uint32_t)prod0;
    uint32_t hi1 = (uint32_t)(prod1 >> 32), lo1 = (uint32_t)prod1;
    uint32_t y0 = hi1 ^ x1 ^ k0;
    uint32_t y2 = hi0 ^ x3 ^ k1;
    x0 = y0;
    x1 = lo1;
    x2 = y2;
    x3 = lo0;
  }
  out[0] = x0;
  out[1] = x1;
  out[2] = x2;
  out[3] = x3;
}

/* One random stream: key = seed, counter = (block, pair, cell, step).
 * A double takes two consecutive 32-bit words (low word first) of the
 * current block; a block holds two doubles. */
typedef struct {
  uint32_t k0, k1;
  uint32_t pair, cell, step;
  uint32_t block;
  uint32_t buf[4];
  int used;
} stream;

static void stream_open(stream *s, uint64_t seed, uint32_t pair, uint32_t cell, uint32_t step) {
  s->k0 = (uint32_t)seed;
  s->k1 = (uint32_t)(seed >> 32);
  s->pair = pair;
  s->cell = cell;
  s->step = step;
  s->block = 0;
  s->used = 4;
}

static uint64_t next_u64(stream *s) {
  if (s->used >= 4) {
    uint32_t ctr[4] = {s->block, s->pair, s->cell, s->step};
    orc_philox4x32_10(s->k0, s->k1, ctr, s->buf);
    s->block += 1;
    s->used = 0;
  }
  uint64_t lo = s->buf[s->used];
  uint64_t hi = s->buf[s->used + 1];
  s->used += 2;
  return (hi << 32) | lo;
}

/* uniform double on [0, 1) with 53 random bits */
static double uniform(stream *s) { return (double)(next_u64(s) >> 11) * 0x1p-53; }

/* ------------------------------------------------------------------ */
/* Deterministic exp / log / pow                                        */
/* ------------------------------------------------------------------ */
static double from_bits(uint64_t b) {
  double d;
  memcpy(&d, &b, 8);
  return d;
}
static uint64_t to_bits(double d) {
  uint64_t b;
  memcpy(&b, &d, 8);
  return b;
}

static const double LN2_HI = 0x1.62e42feep-1;       /* ln 2 with 21 trailing zero bits */
static const double LN2_LO = 0x1.a39ef35793c76p-33; /* ln 2 - LN2_HI */
static const double INV_LN2 = 0x1.71547652b82fep+0;
static const double SQRT2 = 0x1.6a09e667f3bcdp+0;

/* exp(x) = 2^k e^r with k = nearest integer to x/ln2, r = x - k ln2 by a
 * two-part ln2 (Cody-Waite), e^r by its Taylor series to degree 17 in
 * Horner form (|r| <= ln2/2, truncation below 1e-24). */
double orc_detexp(double x) {
  if (x != x) return x;
  if (x > 708.0) return INFINITY;
  if (x < -707.0) return 0.0;
  double kd = floor(x * INV_LN2 + 0.5);
  double r = (x - kd * LN2_HI) - kd * LN2_LO;
  /* coefficients 1/n! for n = 17 .. 0 */
  double p = 1.0 / 355687428096000.0;
  p = p * r + 1.0 / 20922789888000.0;
  p = p * r + 1.0 / 1307674368000.0;
  p = p * r + 1.0 / 87178291200.0;
  p = p * r + 1.0 / 6227020800.0;
  p = p * r + 1.0 / 479001600.0;
  p = p * r + 1.0 / 39916800.0;
  p = p * r + 1.0 / 3628800.0;
  p = p * r + 1.0 / 362880.0;
  p = p * r + 1.0 / 40320.0;
  p = p * r + 1.0 / 5040.0;
  p = p * r + 1.0 / 720.0;
  p = p * r + 1.0 / 120.0;
  p = p * r + 1.0 / 24.0;
  p = p * r + 1.0 / 6.0;
  p = p * r + 0.5;
  p = p * r + 1.0;
  p = p * r + 1.0;
  int k = (int)kd;
  double scale = from_bits((uint64_t)(k + 1023) << 52);
  return p * scale;
}

/* log(x) = e ln2 + log(m), m in (sqrt(1/2), sqrt(2)], with
 * log(m) = 2 atanh(s), s = (m-1)/(m+1), as the odd series
 * 2 s (1 + s^2/3 + s^4/5 + ... + s^22/23). */
double orc_detlog(double x) {
  if (x != x) return x;
  if (x < 0.0) return NAN;
  if (x == 0.0) return -INFINITY;
  if (x == INFINITY) return INFINITY;
  int e = 0;
  uint64_t b = to_bits(x);
  if ((b >> 52) == 0) { /* subnormal */
    x = x * 0x1p54;
    b = to_bits(x);
    e = -54;
  }
  e += (int)((b >> 52) & 0x7ff) - 1023;
  double m = from_bits((b & 0x000fffffffffffffULL) | 0x3ff0000000000000ULL);
  if (m > SQRT2) {
    m = m * 0.5;
    e += 1;
  }
  double s = (m - 1.0) / (m + 1.0);
  double z = s * s;
  double q = 1.0 / 23.0;
  q = q * z + 1.0 / 21.0;
  q = q * z + 1.0 / 19.0;
  q = q * z + 1.0 / 17.0;
  q = q * z + 1.0 / 15.0;
  q = q * z + 1.0 / 13.0;
  q = q * z + 1.0 / 11.0;
  q = q * z + 1.0 / 9.0;
  q = q * z + 1.0 / 7.0;
  q = q * z + 1.0 / 5.0;
  q = q * z + 1.0 / 3.0;
  q = q * z + 1.0;
  double t = s * q;
  double lm = t + t;
  double ed = (double)e;
  return (ed * LN2_LO + lm) + ed * LN2_HI;
}

double orc_detpow(double x, double y) {
  if (x == 0.0) return (y > 0.0) ? 0.0 : ((y == 0.0) ? 1.0 : INFINITY);
  if (x < 0.0) return NAN;
  return orc_detexp(y * orc_detlog(x));
}

/* ------------------------------------------------------------------ */
/* Keyed permutation of [0, n): a Feistel network on Z_m x Z_m with
 * m = ceil(sqrt(n)) and addition modulo m in place of xor (a generalised
 * Feistel cipher, Black & Rogaway 2002), 16 rounds for m <= 8 and 10 rounds
 * above, then cycle walking into [0, n). The round function mixes the right
 * half with the round key using 24-bit factors and maps the 32-bit hash to
 * [0, m) by its high product with m. */
static uint32_t feistel_round(uint32_t r, uint32_t key, uint32_t m) {
  uint32_t h = ((r ^ key) & 0xFFFFFFu) * 0x9E3779u;
  h ^= h >> 15;
  h = (h & 0xFFFFFFu) * 0x85EBCBu;
  h ^= h >> 13;
  return (uint32_t)(((uint64_t)h * (uint64_t)m) >> 32);
}

static uint32_t feistel_side(uint32_t n) {
  uint32_t m = 1;
  while ((uint64_t)m * (uint64_t)m < (uint64_t)n) m += 1;
  return m;
}

static uint32_t feistel_once(uint32_t x, uint32_t m, const uint32_t keys[16]) {
  uint32_t rounds = m <= 8 ? 16 : 10;
  uint32_t left = x / m, right = x % m;
  for (uint32_t r = 0; r < rounds; ++r) {
    uint32_t nl = right;
    uint32_t nr = (left + feistel_round(right, keys[r], m)) % m;
    left = nl;
    right = nr;
  }
  return left * m + right;
}

uint32_t orc_feistel_index(uint32_t n, const uint32_t keys[16], uint32_t i) {
  uint32_t m = feistel_side(n);
  uint32_t y = feistel_once(i, m, keys);
  while (y >= n) y = feistel_once(y, m, keys);
  return y;
}

/* ------------------------------------------------------------------ */
/* Data model                                                            */
/* ------------------------------------------------------------------ */
typedef struct {
  double mass, dref, omega, tref;
  uint32_t n_bend, n_stretch, n_modes;
  double kt[ORC_MAX_MODES];     /* bends: k_B Theta */
  double theta[ORC_MAX_MODES];  /* bends: Theta */
  double *lev[ORC_MAX_MODES];   /* stretches: level energies, index 0..idiss */
  uint32_t idiss[ORC_MAX_MODES];
  double de[ORC_MAX_MODES];     /* stretches: dissociation energy D_e */
  double zpe;
  double formation;
  double p_vib;
  uint32_t zeta_rot;           /* rotational degrees of freedom: 0, 2 or 3 */
  double p_rot;                /* rotational relaxation probability per collision */
  int sampler;                 /* resolved: JOINT, GIBBS or EXACT */
  int concave[ORC_MAX_MODES]; /* level spacings never increase (bends, Morse stretches) */
} species_t;

typedef struct {
  double mr, hm, m_a, m_b, msum, wa, wb, csg, esg, q;
} pair_t;

#define REC_NT 1024
#define REC_TMIN 100.0
#define REC_TMAX 5.0e4

typedef struct {
  int kind;
  int a, b, c, d; /* diss: a -> c + d (b = -1); exch: a + b -> c + d; recomb: a + b -> c (d = -1) */
  uint64_t mask;
  double alpha[ORC_MAX_MODES];
  double steric, ea;
  double dh;   /* sum of formation energies of products minus reactants */
  double zsum; /* dissociation: ZPE_A + ZPE_B + ZPE_C */
  uint32_t n_samp;
  double gamma_rot; /* degree of rotation coupling in the collision energy (Sec. Rotation coupling) */
  double *rec; /* recombination: [third-body species][REC_NT] k_b / <sigma g>_BC  [m^3] */
} reaction_t;

typedef struct {
  uint32_t n, cap;
  double *vx, *vy, *vz;
  uint8_t *sp;
  uint16_t *lvl; /* n x max_modes, row major */
  double *rot;   /* rotational energy [J] */
  double *px, *py, *pz; /* positions [m] (spatial mode) */
  double volume, weight, sgmax, rem;
  /* recombination: running sums of m, m v_x, m v_y, m v_z, m |v|^2 over the
   * cell's particles, from which the step takes the cell temperature */
  double tsum[5];
  uint64_t ctr[ORC_N_CTR];
} cell_t;

struct orc_ctx {
  uint64_t seed;
  uint32_t n_cells, cap_default, step, finalized, loaded;
  uint32_t n_species, n_reactions, max_modes, has_recomb, has_rot;
  uint32_t spatial, nx, ny, nz, periodic; /* spatial mode: box of nx ny nz cells, periodic axes (bits) */
  double len[3];
  /* open faces (bit 2 axis + side) and their reservoir; per (face cell,
   * species) remainder of the expected inflow; particles in and out */
  uint32_t open_faces, n_face_cells;
  double in_flux[ORC_MAX_SPECIES]; /* n_s sqrt(k T / (2 pi m_s)) [m^-2 s^-1] */
  double in_t, in_tv;
  double *in_rem;
  uint64_t flux_in, flux_out;
  double rec_l0, rec_inv_step; /* log(REC_TMIN), (REC_NT - 1) / log(REC_TMAX / REC_TMIN) */
  species_t sp[ORC_MAX_SPECIES];
  reaction_t rx[ORC_MAX_REACTIONS];
  pair_t pr[ORC_MAX_SPECIES][ORC_MAX_SPECIES];
  cell_t *cells;
  int threads; /* OpenMP threads over cells in orc_step (0 or 1: serial) */
};

static void reset_inflow(orc_ctx *o);
static void init_sums(const orc_ctx *o, cell_t *C);

static double mode_energy(const species_t *s, uint32_t m, uint32_t i) {
  if (m < s->n_bend) return ((double)i + 0.5) * s->kt[m];
  return s->lev[m][i];
}

static double vib_energy(const species_t *s, const uint16_t *lvl) {
  double e = 0.0;
  for (uint32_t m = 0; m < s->n_modes; ++m) e = e + mode_energy(s, m, lvl[m]);
  return e;
}

/* ------------------------------------------------------------------ */
/* Context set-up                                                        */
/* ------------------------------------------------------------------ */
int orc_create(uint64_t seed, uint32_t n_cells, const double *cell_volume, const double *cell_weight,
               uint32_t capacity_per_cell, orc_ctx **out) {
  if (!out || n_cells == 0 || !cell_volume || !cell_weight) return E_INVAL;
  orc_ctx *o = (orc_ctx *)calloc(1, sizeof(orc_ctx));
  if (!o) return E_NOMEM;
  o->seed = seed;
  o->n_cells = n_cells;
  o->cap_default = capacity_per_cell;
  o->cells = (cell_t *)calloc(n_cells, sizeof(cell_t));
  if (!o->cells) {
    free(o);
    return E_NOMEM;
  }
  for (uint32_t c = 0; c < n_cells; ++c) {
    if (!(cell_volume[c] > 0.0) || !(cell_weight[c] > 0.0)) {
      free(o->cells);
      free(o);
      return E_INVAL;
    }
    o->cells[c].volume = cell_volume[c];
    o->cells[c].weight = cell_weight[c];
  }
  *out = o;
  return E_OK;
}

static void free_cell(cell_t *c) {
  free(c->vx);
  free(c->vy);
  free(c->vz);
  free(c->sp);
  free(c->lvl);
  free(c->rot);
  free(c->px);
  free(c->py);
  free(c->pz);
  c->vx = c->vy = c->vz = NULL;
  c->sp = NULL;
  c->lvl = NULL;
  c->rot = NULL;
  c->px = c->py = c->pz = NULL;
}

void orc_destroy(orc_ctx *o) {
  if (!o) return;
  for (uint32_t r = 0; r < o->n_reactions; ++r) free(o->rx[r].rec);
  for (uint32_t s = 0; s < o->n_species; ++s)
    for (uint32_t m = 0; m < ORC_MAX_MODES; ++m) free(o->sp[s].lev[m]);
  if (o->cells)
    for (uint32_t c = 0; c < o->n_cells; ++c) free_cell(&o->cells[c]);
  free(o->cells);
  free(o->in_rem);
  free(o);
}

/* Morse (anharmonic) levels, Eq. energy-AHO: E(i) = a (i+1/2) - a x_e (i+1/2)^2
 * with a = h c w_e. Levels are kept while they stay below D_e and still
 * increase; D_e defaults to a / (4 x_e) (chi_e = hc w_e / (4 D_e)). */
static int build_stretch(species_t *s, uint32_t m, double we, double xe, double de,
                         uint32_t n_explicit, const double *explicit_levels) {
  double *lev = (double *)malloc(ORC_MAX_LEVELS * sizeof(double));
  if (!lev) return E_NOMEM;
  uint32_t n = 0;
  if (n_explicit > 0) {
    if (!(de > 0.0)) {
      free(lev);
      return E_INVAL;
    }
    for (uint32_t i = 0; i < n_explicit && i < ORC_MAX_LEVELS; ++i) {
      double e = explicit_levels[i];
      if (!(e < de)) break;
      if (i > 0 && !(e > lev[i - 1])) {
        free(lev);
        return E_INVAL;
      }
      lev[n++] = e;
    }
  } else {
    if (!(we > 0.0) || !(xe >= 0.0)) {
      free(lev);
      return E_INVAL;
    }
    double a = (H_PLANCK * C_LIGHT) * we;
    double ax = a * xe;
    if (!(de > 0.0)) {
      if (!(xe > 0.0)) {
        free(lev);
        return E_INVAL;
      }
      de = a / (4.0 * xe);
    }
    for (uint32_t i = 0; i < ORC_MAX_LEVELS; ++i) {
      double v = (double)i + 0.5;
      double e = (a * v) - ((ax * v) * v);
      if (!(e < de)) break;
      if (i > 0 && !(e > lev[i - 1])) break;
      lev[n++] = e;
    }
  }
  if (n == 0) {
    free(lev);
    return E_INVAL;
  }
  s->lev[m] = lev;
  s->idiss[m] = n - 1;
  s->de[m] = de;
  return E_OK;
}

int orc_add_species(orc_ctx *o, double mass, double dref, double omega, double tref,
                    uint32_t n_bend, const double *theta, uint32_t n_stretch, const double *omega_e,
                    const double *chi_e, const double *de, const uint32_t *n_levels,
                    const double *levels, double formation, double p_vib, int sampler) {
  if (!o || o->finalized) return E_STATE;
  if (o->n_species >= ORC_MAX_SPECIES) return E_INVAL;
  if (!(mass > 0.0) || !(dref > 0.0) || !(tref > 0.0) || !(omega >= 0.5) || !(omega < 1.5)) return E_INVAL;
  if (n_bend + n_stretch > ORC_MAX_MODES) return E_INVAL;
  if (!(p_vib >= 0.0) || !(p_vib <= 1.0)) return E_INVAL;
  species_t *s = &o->sp[o->n_species];
  memset(s, 0, sizeof(*s));
  s->mass = mass;
  s->dref = dref;
  s->omega = omega;
  s->tref = tref;
  s->n_bend = n_bend;
  s->n_stretch = n_stretch;
  s->n_modes = n_bend + n_stretch;
  s->formation = formation;
  s->p_vib = p_vib;
  for (uint32_t j = 0; j < n_bend; ++j) {
    if (!(theta[j] > 0.0)) return E_INVAL;
    s->theta[j] = theta[j];
    s->kt[j] = K_BOLTZ * theta[j];
  }
  const double *lv = levels;
  for (uint32_t j = 0; j < n_stretch; ++j) {
    uint32_t ne = n_levels ? n_levels[j] : 0;
    double dej = de ? de[j] : 0.0;
    int rc = build_stretch(s, n_bend + j, omega_e ? omega_e[j] : 0.0, chi_e ? chi_e[j] : 0.0, dej, ne, lv);
    if (rc) {
      for (uint32_t m = 0; m < ORC_MAX_MODES; ++m) {
        free(s->lev[m]);
        s->lev[m] = NULL;
      }
      return rc;
    }
    if (lv) lv += ne;
  }
  double z = 0.0;
  for (uint32_t m = 0; m < s->n_modes; ++m) z = z + mode_energy(s, m, 0);
  s->zpe = z;
  /* concavity of the level sequence, which the Gibbs proposal relies on */
  for (uint32_t m = 0; m < s->n_modes; ++m) {
    int ok = 1;
    if (m >= s->n_bend)
      for (uint32_t i = 1; i < s->idiss[m]; ++i)
        if (!((s->lev[m][i + 1] - s->lev[m][i]) <= (s->lev[m][i] - s->lev[m][i - 1]))) ok = 0;
    s->concave[m] = ok;
  }
  if (sampler == ORC_SAMPLER_AUTO)
    s->sampler = (s->n_modes >= 2 && s->n_modes <= 4) ? ORC_SAMPLER_JOINT : ORC_SAMPLER_GIBBS;
  else if (sampler == ORC_SAMPLER_JOINT || sampler == ORC_SAMPLER_GIBBS || sampler == ORC_SAMPLER_EXACT)
    s->sampler = sampler;
  else
    return E_INVAL;
  if (s->n_modes > o->max_modes) o->max_modes = s->n_modes;
  o->n_species += 1;
  return E_OK;
}

/* Rotational mode of a species (the paper does not define one): zeta rotational degrees of
 * freedom (0 none, 2 linear, 3 nonlinear rotor), relaxed with probability
 * p_rot per non-reactive collision. Before finalize. */
int orc_set_rotation(orc_ctx *o, uint32_t species, uint32_t zeta, double p_rot) {
  if (!o || o->finalized) return E_STATE;
  if (species >= o->n_species || !(zeta == 0 || zeta == 2 || zeta == 3)) return E_INVAL;
  if (!(p_rot >= 0.0) || !(p_rot <= 1.0)) return E_INVAL;
  o->sp[species].zeta_rot = zeta;
  o->sp[species].p_rot = p_rot;
  if (zeta > 0) o->has_rot = 1;
  return E_OK;
}

/* Degree of rotation coupling gamma in [0, 1] of a dissociation or exchange
 * (Sec. Rotation coupling). Before finalize. */
int orc_set_gamma_rot(orc_ctx *o, uint32_t reaction, double gamma) {
  if (!o || o->finalized) return E_STATE;
  if (reaction >= o->n_reactions || !(gamma >= 0.0) || !(gamma <= 1.0)) return E_INVAL;
  if (o->rx[reaction].kind == ORC_RX_RECOMBINATION && gamma != 0.0) return E_INVAL;
  o->rx[reaction].gamma_rot = gamma;
  return E_OK;
}

/* Spatial mode (not in the paper, whose cases are 0D reservoirs): the cells tile the box [0, lx) x
 * [0, ly) x [0, lz) as an nx x ny x nz grid, cell = ix + nx (iy + ny iz);
 * bit k of periodic makes axis k periodic, else its walls reflect
 * specularly. Every step then moves all particles ballistically, re-bins
 * them by a stable counting sort on the new cell, and collides. Before
 * finalize; every cell's volume must be the grid cell's. */
int orc_set_domain(orc_ctx *o, uint32_t nx, uint32_t ny, uint32_t nz, double lx, double ly, double lz,
                   uint32_t periodic) {
  if (!o || o->finalized) return E_STATE;
  if (nx == 0 || ny == 0 || nz == 0 || (uint64_t)nx * ny * nz != o->n_cells) return E_INVAL;
  if (!(lx > 0.0) || !(ly > 0.0) || !(lz > 0.0) || periodic > 7u) return E_INVAL;
  double vc = ((lx * ly) * lz) / (double)o->n_cells;
  for (uint32_t c = 0; c < o->n_cells; ++c)
    if (fabs(o->cells[c].volume - vc) > 1e-9 * vc) return E_INVAL;
  o->spatial = 1;
  o->nx = nx;
  o->ny = ny;
  o->nz = nz;
  o->len[0] = lx;
  o->len[1] = ly;
  o->len[2] = lz;
  o->periodic = periodic;
  return E_OK;
}

/* grid index along axis k of coordinate x: floor(x / (L_k / n_k)), clamped */
static uint32_t axis_index(const orc_ctx *o, int k, double x) {
  uint32_t n = k == 0 ? o->nx : (k == 1 ? o->ny : o->nz);
  double d = o->len[k] / (double)n;
  double f = floor(x / d);
  if (!(f >= 0.0)) return 0;
  if (f >= (double)n) return n - 1;
  return (uint32_t)f;
}

static uint32_t cell_of(const orc_ctx *o, double x, double y, double z) {
  return axis_index(o, 0, x) + o->nx * (axis_index(o, 1, y) + o->ny * axis_index(o, 2, z));
}

/* ballistic move of one coordinate over dt with the axis' boundary:
 * periodic wraps into [0, L); a specular face reflects (x < 0: -x, x > L:
 * 2L - x, velocity reversed) until inside [0, L]; crossing an open face
 * (x < 0 with the face at 0 open, x > L with the face at L open) ends the
 * move: returns 1, the particle leaves the box */
static int move_axis(double *x, double *v, double dt, double len, int periodic, int open_lo, int open_hi) {
  double y = *x + *v * dt;
  if (periodic) {
    while (y < 0.0) y = y + len;
    while (y >= len) y = y - len;
  } else {
    for (;;) {
      if (y < 0.0) {
        if (open_lo) return 1;
        y = -y;
        *v = -*v;
      } else if (y > len) {
        if (open_hi) return 1;
        y = (len + len) - y;
        *v = -*v;
      } else {
        break;
      }
    }
  }
  *x = y;
  return 0;
}

/* move of one particle on all three axes; 1 if it leaves through an open face */
static int move_particle(const orc_ctx *o, double *x, double *y, double *z, double *vx, double *vy, double *vz,
                         double dt) {
  const uint32_t f = o->open_faces;
  if (move_axis(x, vx, dt, o->len[0], (int)(o->periodic & 1u), (int)(f & 1u), (int)((f >> 1) & 1u))) return 1;
  if (move_axis(y, vy, dt, o->len[1], (int)((o->periodic >> 1) & 1u), (int)((f >> 2) & 1u), (int)((f >> 3) & 1u)))
    return 1;
  return move_axis(z, vz, dt, o->len[2], (int)((o->periodic >> 2) & 1u), (int)((f >> 4) & 1u), (int)((f >> 5) & 1u));
}

/* cells per axis */
static uint32_t axis_cells(const orc_ctx *o, int k) { return k == 0 ? o->nx : (k == 1 ? o->ny : o->nz); }

/* the two axes tangential to face f, in increasing order, and the number of
 * face cells (face cell j = i_a + n_a i_b) */
static void face_axes(const orc_ctx *o, uint32_t f, int *a, int *b, uint32_t *size) {
  int k = (int)(f >> 1);
  *a = k == 0 ? 1 : 0;
  *b = k == 2 ? 1 : 2;
  *size = axis_cells(o, *a) * axis_cells(o, *b);
}

/* Surface-flux boundaries (spatial mode; not in the paper, whose cases are
 * 0D reservoirs). Face f = 2 k + side lies on axis k at coordinate 0 (side
 * 0) or L_k (side 1); bit f of open makes it open. A particle whose move
 * crosses an open face leaves the box. Every step, after the move, each
 * open face admits from a resting Maxwellian reservoir of number densities
 * n_s at t_trans (translation and rotation) and t_vib: face cell j of face f
 * gets floor(x) particles of species s, x = ((F_s A) dt) / F_N + rem, with
 * the one-sided flux F_s = n_s sqrt(k T / (2 pi m_s)), A the face cell's area,
 * F_N the weight of the cell behind it and rem the fraction carried from the
 * previous step. Axes with an open face must not be periodic. */
int orc_set_inflow(orc_ctx *o, uint32_t open, const double *n_s, double t_trans, double t_vib) {
  if (!o || !o->spatial || !o->finalized) return E_STATE;
  if (open > 63u || !n_s || !(t_trans > 0.0) || !(t_vib > 0.0) || !isfinite(t_trans) || !isfinite(t_vib))
    return E_INVAL;
  for (int k = 0; k < 3; ++k)
    if (((o->periodic >> k) & 1u) && ((open >> (2 * k)) & 3u)) return E_INVAL;
  for (uint32_t s = 0; s < o->n_species; ++s)
    if (!(n_s[s] >= 0.0) || !isfinite(n_s[s])) return E_INVAL;
  uint32_t total = 0;
  for (uint32_t f = 0; f < 6; ++f) {
    int a, b;
    uint32_t size;
    face_axes(o, f, &a, &b, &size);
    total += size;
  }
  double *rem = (double *)calloc((size_t)total * o->n_species, sizeof(double));
  if (!rem) return E_NOMEM;
  free(o->in_rem);
  o->in_rem = rem;
  o->n_face_cells = total;
  o->open_faces = open;
  o->in_t = t_trans;
  o->in_tv = t_vib;
  for (uint32_t s = 0; s < o->n_species; ++s)
    o->in_flux[s] = n_s[s] * sqrt((K_BOLTZ * t_trans) / ((2.0 * PI_D) * o->sp[s].mass));
  return E_OK;
}

int orc_flux_counts(const orc_ctx *o, uint64_t *out) {
  if (!o || !out) return E_INVAL;
  out[0] = o->flux_in;
  out[1] = o->flux_out;
  return E_OK;
}

int orc_add_reaction(orc_ctx *o, int kind, const int32_t reactant[2], const int32_t product[2],
                     uint64_t stretch_mask, const double *alpha, double steric, double ea, uint32_t n_samp) {
  if (!o || o->finalized) return E_STATE;
  if (o->n_reactions >= ORC_MAX_REACTIONS) return E_INVAL;
  int ns = (int)o->n_species;
  reaction_t *r = &o->rx[o->n_reactions];
  memset(r, 0, sizeof(*r));
  r->kind = kind;
  if (kind == ORC_RX_DISSOCIATION) {
    int a = reactant[0], c = product[0], d = product[1];
    if (a < 0 || a >= ns || c < 0 || c >= ns || d < 0 || d >= ns) return E_INVAL;
    const species_t *A = &o->sp[a];
    if (A->n_stretch == 0) return E_INVAL;
    if (stretch_mask == 0 || (A->n_stretch < 64 && (stretch_mask >> A->n_stretch) != 0)) return E_INVAL;
    double msum = o->sp[c].mass + o->sp[d].mass;
    if (fabs(msum - A->mass) > 1e-9 * A->mass) return E_INVAL;
    r->a = a;
    r->b = -1;
    r->c = c;
    r->d = d;
    r->mask = stretch_mask;
    r->dh = (o->sp[c].formation + o->sp[d].formation) - A->formation;
    r->zsum = (A->zpe + o->sp[c].zpe) + o->sp[d].zpe;
  } else if (kind == ORC_RX_EXCHANGE) {
    int a = reactant[0], b = reactant[1], c = product[0], d = product[1];
    if (a < 0 || a >= ns || b < 0 || b >= ns || c < 0 || c >= ns || d < 0 || d >= ns) return E_INVAL;
    if (!(steric >= 0.0) || !(steric <= 1.0) || !(ea >= 0.0)) return E_INVAL;
    double m_in = o->sp[a].mass + o->sp[b].mass, m_out = o->sp[c].mass + o->sp[d].mass;
    if (fabs(m_in - m_out) > 1e-9 * m_in) return E_INVAL;
    r->a = a;
    r->b = b;
    r->c = c;
    r->d = d;
    for (uint32_t m = 0; m < o->sp[a].n_modes; ++m) {
      double al = alpha ? alpha[m] : 0.0;
      if (!(al >= 0.0) || !(al <= 1.0)) return E_INVAL;
      r->alpha[m] = al;
    }
    r->steric = steric;
    r->ea = ea;
    r->dh = (o->sp[c].formation + o->sp[d].formation) - (o->sp[a].formation + o->sp[b].formation);
  } else if (kind == ORC_RX_RECOMBINATION) {
    /* B + C (+M) -> A (+M): reactant = {B, C}, product[0] = A; stretch_mask names
     * the bond(s) of A whose dissociation this reverses (D_e of the first one) */
    int b = reactant[0], c = reactant[1], a = product[0];
    if (a < 0 || a >= ns || b < 0 || b >= ns || c < 0 || c >= ns || b == c) return E_INVAL;
    const species_t *A = &o->sp[a];
    if (A->n_stretch == 0 || stretch_mask == 0 || (A->n_stretch < 64 && (stretch_mask >> A->n_stretch) != 0))
      return E_INVAL;
    double msum = o->sp[b].mass + o->sp[c].mass;
    if (fabs(msum - A->mass) > 1e-9 * A->mass) return E_INVAL;
    r->a = b;
    r->b = c;
    r->c = a;
    r->d = -1;
    r->mask = stretch_mask;
    r->dh = A->formation - (o->sp[b].formation + o->sp[c].formation);
    r->n_samp = n_samp ? n_samp : 1000;
  } else {
    return E_INVAL;
  }
  o->n_reactions += 1;
  return E_OK;
}

/* VHS pair constants (Bird): sigma g = C (g^2)^(1-w), with
 * C = pi d^2 (2 k T_ref / m_r)^(w - 1/2) / Gamma(5/2 - w); mixed-pair d, w and
 * T_ref are the means of both species. LB exponent xi_rel/2 - 1 = 3/2 - w. */
static void build_pair(orc_ctx *o, uint32_t a, uint32_t b) {
  const species_t *A = &o->sp[a], *B = &o->sp[b];
  pair_t *p = &o->pr[a][b];
  double msum = A->mass + B->mass;
  double mr = (A->mass * B->mass) / msum;
  double w = (A->omega + B->omega) * 0.5;
  double d = (A->dref + B->dref) * 0.5;
  double tr = (A->tref + B->tref) * 0.5;
  double base = ((2.0 * K_BOLTZ) * tr) / mr;
  p->mr = mr;
  p->hm = 0.5 * mr;
  p->m_a = A->mass;
  p->m_b = B->mass;
  p->msum = msum;
  p->wa = B->mass / msum;
  p->wb = A->mass / msum;
  p->csg = ((PI_D * (d * d)) * pow(base, w - 0.5)) / tgamma(2.5 - w);
  p->esg = 1.0 - w;
  p->q = 1.5 - w;
}

/* ------------------------------------------------------------------ */
/* Recombination rate tables (Sec. "Recombination reactions")            */
/* ------------------------------------------------------------------ */

/* Regularized upper incomplete gamma Q(a, x), x > 0: series for x < a + 1,
 * Lentz continued fraction otherwise (Press et al., Numerical Recipes 6.2). */
static double gamma_q(double a, double x) {
  if (!(x > 0.0)) return 1.0;
  double lpre = -x + a * log(x) - lgamma(a);
  if (x < a + 1.0) {
    double ap = a, del = 1.0 / a, sum = del;
    for (int n = 1; n <= 1000; ++n) {
      ap = ap + 1.0;
      del = del * (x / ap);
      sum = sum + del;
      if (fabs(del) < fabs(sum) * 1e-17) break;
    }
    return 1.0 - sum * exp(lpre);
  }
  const double tiny = 1e-300;
  double bb = x + 1.0 - a, c = 1.0 / tiny, d = 1.0 / bb, h = d;
  for (int i = 1; i <= 1000; ++i) {
    double an = -(double)i * ((double)i - a);
    bb = bb + 2.0;
    d = an * d + bb;
    if (fabs(d) < tiny) d = tiny;
    c = bb + an / c;
    if (fabs(c) < tiny) c = tiny;
    d = 1.0 / d;
    double del = d * c;
    h = h * del;
    if (fabs(del - 1.0) < 1e-17) break;
  }
  return exp(lpre) * h;
}

/* vibrational partition sum of a species, energies from its ground state */
static double q_vib(const species_t *s, double t) {
  double q = 1.0;
  for (uint32_t m = 0; m < s->n_bend; ++m) q = q * (1.0 / (1.0 - exp(-s->theta[m] / t)));
  for (uint32_t m = s->n_bend; m < s->n_modes; ++m) {
    double z = 0.0;
    for (uint32_t i = 0; i <= s->idiss[m]; ++i) z = z + exp(-(s->lev[m][i] - s->lev[m][0]) / (K_BOLTZ * t));
    q = q * z;
  }
  return q;
}

/* forward probability P(T) of the recombination section with the
 * Whitten-Rabinovich density of states at n_samp evenly spaced energies */
static double wr_probability(const species_t *A, double de, double omega, uint32_t n_samp, double t) {
  uint32_t l = A->n_modes;
  double nu_sum = 0.0, nu2_sum = 0.0;
  for (uint32_t m = 0; m < l; ++m) {
    double nu = (m < A->n_bend) ? (K_BOLTZ * A->theta[m]) / H_PLANCK : (A->lev[m][1] - A->lev[m][0]) / H_PLANCK;
    nu_sum = nu_sum + nu;
    nu2_sum = nu2_sum + nu * nu;
  }
  double ez = 0.5 * H_PLANCK * nu_sum;
  double lm1 = (double)l - 1.0;
  double beta = (lm1 * lm1 * nu2_sum) / ((double)l * (nu_sum * nu_sum));
  double num = 0.0, den = 0.0;
  for (uint32_t i = 1; i <= n_samp; ++i) {
    double e = (double)(i - 1) * de / (double)(n_samp - 1);
    double r = e / ez;
    double omg = (r >= 1.0) ? pow(10.0, -1.0506 * pow(r, 0.25)) : 1.0 / (5.0 * r + 2.73 * sqrt(r) + 3.51);
    double aw = 1.0 - beta * omg;
    double rho = pow(e + aw * ez, lm1);
    double w = rho * exp(-e / (K_BOLTZ * t));
    num = num + gamma_q(2.5 - omega, (de - e) / (K_BOLTZ * t)) * w;
    den = den + w;
  }
  return den > 0.0 ? num / den : 0.0;
}

/* Equilibrium constant of A <-> B + C [m^-3] from partition functions per
 * unit volume: translation (2 pi m k T / h^2)^(3/2) of each species and the
 * vibrational sums from the ground state (no rotation is modelled), with the
 * ground-to-ground energy change dE0 = (h_B + ZPE_B + h_C + ZPE_C) - (h_A +
 * ZPE_A). Expression order: ((((2 pi k T / h^2)^(3/2) (m_B m_C / m_A)^(3/2))
 * (Q_B Q_C / Q_A)) exp(-dE0 / kT)). */
static double equilibrium_constant(const orc_ctx *o, const reaction_t *R, double t) {
  const species_t *B = &o->sp[R->a], *C = &o->sp[R->b], *A = &o->sp[R->c];
  double de0 = ((B->formation + B->zpe) + (C->formation + C->zpe)) - (A->formation + A->zpe);
  double ktr = (2.0 * PI_D * K_BOLTZ * t) / (H_PLANCK * H_PLANCK);
  return pow(ktr, 1.5) * pow((B->mass * C->mass) / A->mass, 1.5) * ((q_vib(B, t) * q_vib(C, t)) / q_vib(A, t)) *
         exp(-de0 / (K_BOLTZ * t));
}

/* Maxwellian mean of the VHS sigma g of a pair with mean diameter d,
 * exponent w and reference temperature tr, reduced mass mred, at t:
 * 2 d^2 sqrt(2 pi k tr / mred) (t / tr)^(1 - w). */
static double mean_sigma_g(double d, double w, double tr, double mred, double t) {
  return 2.0 * (d * d) * sqrt((2.0 * PI_D * K_BOLTZ * tr) / mred) * pow(t / tr, 1.0 - w);
}

/* dissociation energy of the recombining bond: D_e of A's first listed stretch */
static double recombination_de(const orc_ctx *o, const reaction_t *R) {
  const species_t *A = &o->sp[R->c];
  uint32_t j = 0;
  while (!((R->mask >> j) & 1ULL)) ++j;
  return A->de[A->n_bend + j];
}

/* Forward rate coefficient of A + M -> B + C + M [m^3/s]: the paper's
 * forward probability P(T) (Whitten-Rabinovich; it depends on the third body
 * only through the A-M VHS exponent) times the Maxwellian collision rate
 * coefficient of A with M, halved for identical partners (M = A). The
 * probability p is passed in so that the table builder evaluates it once
 * per exponent. */
static double forward_rate(const orc_ctx *o, const reaction_t *R, uint32_t m, double p, double t) {
  const species_t *A = &o->sp[R->c], *M = &o->sp[m];
  double w = (A->omega + M->omega) * 0.5, d = (A->dref + M->dref) * 0.5, tr = (A->tref + M->tref) * 0.5;
  double mred = (A->mass * M->mass) / (A->mass + M->mass);
  double delta = ((uint32_t)R->c == m) ? 2.0 : 1.0;
  return p * ((2.0 * (d * d)) / delta) * sqrt((2.0 * PI_D * K_BOLTZ * tr) / mred) * pow(t / tr, 1.0 - w);
}

static double forward_probability(const orc_ctx *o, const reaction_t *R, uint32_t m, double t) {
  const species_t *A = &o->sp[R->c], *M = &o->sp[m];
  return wr_probability(A, recombination_de(o, R), (A->omega + M->omega) * 0.5, R->n_samp, t);
}

/* Table of the per-collision recombination factor k_b / <sigma g>_BC
 * (k_b = k_f / K_eq) per third-body species on the log-spaced nodes. */
static int build_recombination(orc_ctx *o, reaction_t *R) {
  const species_t *B = &o->sp[R->a], *C = &o->sp[R->b], *A = &o->sp[R->c];
  const pair_t *pbc = &o->pr[R->a][R->b];
  double w_bc = 1.0 - pbc->esg;
  double d_bc = (B->dref + C->dref) * 0.5, t_bc = (B->tref + C->tref) * 0.5;
  R->rec = (double *)calloc((size_t)o->n_species * REC_NT, sizeof(double));
  if (!R->rec) return E_NOMEM;
  for (uint32_t i = 0; i < REC_NT; ++i) {
    double t = exp(o->rec_l0 + (double)i / o->rec_inv_step);
    double sg_bc = mean_sigma_g(d_bc, w_bc, t_bc, pbc->mr, t);
    double keq = equilibrium_constant(o, R, t);
    double p_w = -1.0, p = 0.0;
    for (uint32_t m = 0; m < o->n_species; ++m) {
      double w = (A->omega + o->sp[m].omega) * 0.5;
      if (w != p_w) {
        p = forward_probability(o, R, m, t);
        p_w = w;
      }
      double v = (forward_rate(o, R, m, p, t) / keq) / sg_bc;
      R->rec[(size_t)m * REC_NT + i] = (v == v && v >= 0.0) ? v : 0.0;
    }
  }
  return E_OK;
}

static const reaction_t *recombination_of(const orc_ctx *o, uint32_t reaction) {
  if (!o || reaction >= o->n_reactions || o->rx[reaction].kind != ORC_RX_RECOMBINATION) return NULL;
  return &o->rx[reaction];
}

double orc_equilibrium_constant(const orc_ctx *o, uint32_t reaction, double t) {
  const reaction_t *R = recombination_of(o, reaction);
  return R && t > 0.0 ? equilibrium_constant(o, R, t) : -1.0;
}

double orc_forward_rate(const orc_ctx *o, uint32_t reaction, uint32_t third, double t) {
  const reaction_t *R = recombination_of(o, reaction);
  if (!R || third >= o->n_species || !(t > 0.0)) return -1.0;
  return forward_rate(o, R, third, forward_probability(o, R, third, t), t);
}

double orc_forward_probability(const orc_ctx *o, uint32_t reaction, uint32_t third, double t) {
  const reaction_t *R = recombination_of(o, reaction);
  if (!R || third >= o->n_species || !(t > 0.0)) return -1.0;
  return forward_probability(o, R, third, t);
}

double orc_rec_node_temperature(const orc_ctx *o, uint32_t i) {
  return exp(o->rec_l0 + (double)i / o->rec_inv_step);
}

int orc_finalize(orc_ctx *o) {
  if (!o || o->finalized) return E_STATE;
  if (o->n_species == 0) return E_INVAL;
  for (uint32_t a = 0; a < o->n_species; ++a)
    for (uint32_t b = 0; b < o->n_species; ++b) build_pair(o, a, b);
  o->rec_l0 = log(REC_TMIN);
  o->rec_inv_step = (double)(REC_NT - 1) / log(REC_TMAX / REC_TMIN);
  for (uint32_t r = 0; r < o->n_reactions; ++r) {
    if (o->rx[r].kind != ORC_RX_RECOMBINATION) continue;
    o->has_recomb = 1;
    int rc = build_recombination(o, &o->rx[r]);
    if (rc) return rc;
  }
  o->finalized = 1;
  return E_OK;
}

double orc_gamma_q(double a, double x) { return gamma_q(a, x); }

/* normalised Whitten-Rabinovich density of states of species s at energy e
 * above its ground state: [e + a(e) E_z]^(l-1) / ((l-1)! prod h nu_k) */
double orc_wr_rho(const orc_ctx *o, uint32_t species, double e) {
  const species_t *A = &o->sp[species];
  uint32_t l = A->n_modes;
  double nu_sum = 0.0, nu2_sum = 0.0, prod = 1.0;
  for (uint32_t m = 0; m < l; ++m) {
    double nu = (m < A->n_bend) ? (K_BOLTZ * A->theta[m]) / H_PLANCK : (A->lev[m][1] - A->lev[m][0]) / H_PLANCK;
    nu_sum = nu_sum + nu;
    nu2_sum = nu2_sum + nu * nu;
    prod = prod * (H_PLANCK * nu);
  }
  double ez = 0.5 * H_PLANCK * nu_sum;
  double lm1 = (double)l - 1.0;
  double beta = (lm1 * lm1 * nu2_sum) / ((double)l * (nu_sum * nu_sum));
  double r = e / ez;
  double omg = (r >= 1.0) ? pow(10.0, -1.0506 * pow(r, 0.25)) : 1.0 / (5.0 * r + 2.73 * sqrt(r) + 3.51);
  double aw = 1.0 - beta * omg;
  return pow(e + aw * ez, lm1) / (tgamma((double)l) * prod);
}

double orc_wr_probability(const orc_ctx *o, uint32_t species, double de, double omega, uint32_t n_samp, double t) {
  return wr_probability(&o->sp[species], de, omega, n_samp, t);
}

double orc_q_vib(const orc_ctx *o, uint32_t species, double t) { return q_vib(&o->sp[species], t); }

/* Forward probability of Eq. recomb-correct, summed over every combination
 * of vibrational levels of A: P(T) = sum_i Q(a, (D_e - S_i)/kT)
 * exp(-S_i/kT) / sum_i exp(-S_i/kT), S_i the energy of combination i above
 * the ground level (sum over modes of E_m(j) - E_m(0)), a = 5/2 - omega, Q the
 * regularized upper incomplete gamma with Q = 1 for a non-positive argument.
 * Bends are infinite harmonic ladders, stretches run over 0..i_diss.
 * Combinations below D_e are enumerated one by one (depth-first over the
 * modes in order); every combination at or above D_e has Q = 1, and those
 * are summed in closed form where the enumeration first crosses D_e: at mode
 * m with partial energy S_p, the levels j' >= j of m that cross, times all
 * levels of the later modes, give exp(-S_p/kT) sum_{j'>=j} exp(-e_m(j')/kT)
 * prod_{m'>m} Z_m'. No term is subtracted, so small P keep full precision. */
static double rec_zmode(const species_t *s, uint32_t m, double beta) {
  if (m < s->n_bend) return 1.0 / (1.0 - exp(-(beta * s->kt[m])));
  double z = 0.0;
  for (uint32_t i = 0; i <= s->idiss[m]; ++i) z = z + exp(-(beta * (s->lev[m][i] - s->lev[m][0])));
  return z;
}

static double rec_exact_walk(const species_t *s, uint32_t m, double sp, double de, double a, double beta,
                             const double *zrest) {
  if (m == s->n_modes) return gamma_q(a, beta * (de - sp)) * exp(-(beta * sp));
  double total = 0.0;
  for (uint32_t j = 0;; ++j) {
    if (m >= s->n_bend && j > s->idiss[m]) break; /* stretch ladder ends below D_e */
    double e = mode_energy(s, m, j) - mode_energy(s, m, 0);
    double sj = sp + e;
    if (!(sj < de)) {
      /* levels j.. of mode m cross D_e: closed form over them and the later modes */
      double tail;
      if (m < s->n_bend) {
        tail = exp(-(beta * sj)) / (1.0 - exp(-(beta * s->kt[m])));
      } else {
        tail = 0.0;
        for (uint32_t k = j; k <= s->idiss[m]; ++k)
          tail = tail + exp(-(beta * (sp + (mode_energy(s, m, k) - mode_energy(s, m, 0)))));
      }
      total = total + tail * zrest[m + 1];
      break;
    }
    total = total + rec_exact_walk(s, m + 1, sj, de, a, beta, zrest);
  }
  return total;
}

double orc_rec_exact_probability(const orc_ctx *o, uint32_t species, double de, double omega, double t) {
  if (!o || species >= o->n_species || !(t > 0.0) || !(de > 0.0)) return -1.0;
  const species_t *s = &o->sp[species];
  double beta = 1.0 / (K_BOLTZ * t);
  double zrest[ORC_MAX_MODES + 1];
  zrest[s->n_modes] = 1.0;
  for (uint32_t m = s->n_modes; m-- > 0;) zrest[m] = zrest[m + 1] * rec_zmode(s, m, beta);
  double num = rec_exact_walk(s, 0, 0.0, de, 2.5 - omega, beta, zrest);
  return num / zrest[0];
}

/* per-collision recombination probability factor at the cell temperature,
 * linear in log T between table nodes */
static double rec_lookup(const orc_ctx *o, const reaction_t *R, uint32_t m, double t) {
  const double *tab = R->rec + (size_t)m * REC_NT;
  if (!(t > 0.0)) return tab[0];
  double u = (orc_detlog(t) - o->rec_l0) * o->rec_inv_step;
  if (!(u > 0.0)) return tab[0];
  if (!(u < (double)(REC_NT - 1))) return tab[REC_NT - 1];
  double fi = floor(u);
  uint32_t i = (uint32_t)fi;
  double f = u - fi;
  return tab[i] + f * (tab[i + 1] - tab[i]);
}

double orc_rec_factor(const orc_ctx *o, uint32_t reaction, uint32_t third, double t) {
  if (!o || reaction >= o->n_reactions || o->rx[reaction].kind != ORC_RX_RECOMBINATION || third >= o->n_species)
    return -1.0;
  return rec_lookup(o, &o->rx[reaction], third, t);
}

int orc_rec_table(const orc_ctx *o, uint32_t reaction, double *out) {
  if (!o || reaction >= o->n_reactions || o->rx[reaction].kind != ORC_RX_RECOMBINATION) return E_INVAL;
  memcpy(out, o->rx[reaction].rec, sizeof(double) * o->n_species * REC_NT);
  return REC_NT;
}

/* ------------------------------------------------------------------ */
/* Particle storage                                                      */
/* ------------------------------------------------------------------ */
static int alloc_cell(orc_ctx *o, cell_t *c, uint32_t cap) {
  free_cell(c);
  uint32_t mm = o->max_modes ? o->max_modes : 1;
  c->cap = cap;
  c->n = 0;
  c->vx = (double *)calloc(cap ? cap : 1, sizeof(double));
  c->vy = (double *)calloc(cap ? cap : 1, sizeof(double));
  c->vz = (double *)calloc(cap ? cap : 1, sizeof(double));
  c->sp = (uint8_t *)calloc(cap ? cap : 1, 1);
  c->lvl = (uint16_t *)calloc((size_t)(cap ? cap : 1) * mm, sizeof(uint16_t));
  c->rot = (double *)calloc(cap ? cap : 1, sizeof(double));
  if (!c->vx || !c->vy || !c->vz || !c->sp || !c->lvl || !c->rot) return E_NOMEM;
  if (o->spatial) {
    c->px = (double *)calloc(cap ? cap : 1, sizeof(double));
    c->py = (double *)calloc(cap ? cap : 1, sizeof(double));
    c->pz = (double *)calloc(cap ? cap : 1, sizeof(double));
    if (!c->px || !c->py || !c->pz) return E_NOMEM;
  }
  return E_OK;
}

static uint32_t default_capacity(const orc_ctx *o, uint32_t n) {
  if (o->cap_default) return o->cap_default;
  return n + n / 4 + 32;
}

/* initial (sigma g)_max: an upper bound of sigma g over the cell's pairs,
 * using |v_p - v_q|^2 <= 4 max|v|^2 and the species present */
static void init_sgmax(orc_ctx *o, cell_t *c) {
  double vmax2 = 0.0;
  int present[ORC_MAX_SPECIES] = {0};
  for (uint32_t i = 0; i < c->n; ++i) {
    double v2 = (c->vx[i] * c->vx[i] + c->vy[i] * c->vy[i]) + c->vz[i] * c->vz[i];
    if (v2 > vmax2) vmax2 = v2;
    present[c->sp[i]] = 1;
  }
  double g2 = 4.0 * vmax2;
  double best = 0.0;
  if (g2 > 0.0) {
    for (uint32_t a = 0; a < o->n_species; ++a) {
      if (!present[a]) continue;
      for (uint32_t b = 0; b < o->n_species; ++b) {
        if (!present[b]) continue;
        double sg = o->pr[a][b].csg * orc_detpow(g2, o->pr[a][b].esg);
        if (sg > best) best = sg;
      }
    }
  }
  c->sgmax = best;
  c->rem = 0.0;
}

static int check_particle(const orc_ctx *o, uint32_t sp, const double *v, const uint16_t *lvl) {
  if (sp >= o->n_species) return E_INVAL;
  if (!isfinite(v[0]) || !isfinite(v[1]) || !isfinite(v[2])) return E_NONFINITE;
  const species_t *s = &o->sp[sp];
  for (uint32_t m = 0; m < o->max_modes; ++m) {
    if (m >= s->n_modes) {
      if (lvl[m] != 0) return E_LEVEL;
    } else if (m >= s->n_bend && lvl[m] > s->idiss[m]) {
      return E_LEVEL;
    }
  }
  return E_OK;
}

/* Stable placement of particles into their cells (a counting sort by cell). */
int orc_load(orc_ctx *o, uint64_t n, const uint32_t *cell, const uint8_t *species, const double *vel,
             const uint16_t *levels, const double *rot, const double *pos) {
  if (!o || !o->finalized) return E_STATE;
  uint32_t mm = o->max_modes;
  uint32_t *count = (uint32_t *)calloc(o->n_cells, sizeof(uint32_t));
  if (!count) return E_NOMEM;
  for (uint64_t i = 0; i < n; ++i) {
    if (cell[i] >= o->n_cells) {
      free(count);
      return E_INVAL;
    }
    int rc = check_particle(o, species[i], vel + 3 * i, levels + (size_t)i * mm);
    if (!rc && rot && !(rot[i] >= 0.0 && isfinite(rot[i]) && (rot[i] == 0.0 || o->sp[species[i]].zeta_rot > 0)))
      rc = E_INVAL;
    if (!rc && o->spatial) {
      /* positions inside the box and in the particle's cell */
      if (!pos) rc = E_INVAL;
      for (int k = 0; !rc && k < 3; ++k)
        if (!(pos[3 * i + k] >= 0.0) || !(pos[3 * i + k] <= o->len[k])) rc = E_INVAL;
      if (!rc && cell_of(o, pos[3 * i], pos[3 * i + 1], pos[3 * i + 2]) != cell[i]) rc = E_INVAL;
    }
    if (rc) {
      free(count);
      return rc;
    }
    count[cell[i]] += 1;
  }
  for (uint32_t c = 0; c < o->n_cells; ++c) {
    uint32_t cap = default_capacity(o, count[c]);
    if (count[c] > cap) {
      free(count);
      return E_CAPACITY;
    }
    int rc = alloc_cell(o, &o->cells[c], cap);
    if (rc) {
      free(count);
      return rc;
    }
    memset(o->cells[c].ctr, 0, sizeof(o->cells[c].ctr));
  }
  free(count);
  for (uint64_t i = 0; i < n; ++i) {
    cell_t *c = &o->cells[cell[i]];
    uint32_t j = c->n++;
    c->vx[j] = vel[3 * i];
    c->vy[j] = vel[3 * i + 1];
    c->vz[j] = vel[3 * i + 2];
    c->sp[j] = species[i];
    c->rot[j] = rot ? rot[i] : 0.0;
    if (o->spatial) {
      c->px[j] = pos[3 * i];
      c->py[j] = pos[3 * i + 1];
      c->pz[j] = pos[3 * i + 2];
    }
    for (uint32_t m = 0; m < mm; ++m) c->lvl[(size_t)j * mm + m] = levels[(size_t)i * mm + m];
  }
  for (uint32_t c = 0; c < o->n_cells; ++c) {
    init_sgmax(o, &o->cells[c]);
    init_sums(o, &o->cells[c]);
  }
  o->step = 0;
  o->loaded = 1;
  reset_inflow(o);
  return E_OK;
}

/* Maxwellian components by Marsaglia's polar method (two normals per accepted point). */
static void polar_normals(stream *st, double *n1, double *n2) {
  double x, y, s;
  for (;;) {
    x = 2.0 * uniform(st) - 1.0;
    y = 2.0 * uniform(st) - 1.0;
    s = x * x + y * y;
    if (s < 1.0 && s > 0.0) break;
  }
  double f = sqrt((-2.0 * orc_detlog(s)) / s);
  *n1 = x * f;
  *n2 = y * f;
}

/* Internal state of a molecule drawn at T_vib (levels) and T_rot (rotational
 * energy), the thermal initial state's sampler: levels of every mode in
 * order, then the rotational energy. */
static void sample_internal(const species_t *S, stream *st, double t_vib, double t_rot, uint16_t *lv, uint32_t mm,
                            double *rot) {
  for (uint32_t m = 0; m < mm; ++m) lv[m] = 0;
  for (uint32_t m = 0; m < S->n_modes; ++m) {
    if (m < S->n_bend) {
      double r = 1.0 - uniform(st);
      double t = -orc_detlog(r);
      double fi = floor(t * (t_vib / S->theta[m]));
      if (fi > 65535.0) fi = 65535.0;
      lv[m] = (uint16_t)fi;
    } else {
      uint32_t top = S->idiss[m];
      double kt = K_BOLTZ * t_vib;
      for (;;) {
        double u = uniform(st);
        uint32_t i = (uint32_t)floor(u * (double)(top + 1));
        if (i > top) i = top;
        double u2 = uniform(st);
        double x = (S->lev[m][i] - S->lev[m][0]) / kt;
        if (u2 < orc_detexp(-x)) {
          lv[m] = (uint16_t)i;
          break;
        }
      }
    }
  }
  *rot = 0.0;
  if (S->zeta_rot > 0) {
    double g = -orc_detlog(1.0 - uniform(st));
    if (S->zeta_rot == 3) {
      double z1, z2;
      polar_normals(st, &z1, &z2);
      g = g + 0.5 * (z1 * z1);
    }
    *rot = (K_BOLTZ * t_rot) * g;
  }
}

/* a new particle state starts the inflow remainders and the flux counts afresh */
static void reset_inflow(orc_ctx *o) {
  if (o->in_rem) memset(o->in_rem, 0, (size_t)o->n_face_cells * o->n_species * sizeof(double));
  o->flux_in = 0;
  o->flux_out = 0;
}

/* Thermal initial state. Rotational energy (species with a rotor, after the
 * levels): Boltzmann at T_rot = T_trans, Gamma(zeta/2, k T): zeta = 2 takes
 * -ln(1 - u), zeta = 3 adds half the square of one polar normal. Position
 * (spatial mode, last): uniform in the cell, one draw per axis.
 * Velocities: Maxwellian at T_trans. Bends: the floor
 * form of the initialization section (i = floor(-ln r T_vib / Theta), r in (0,1]).
 * Stretches: uniform proposal over 0..i_diss accepted with
 * exp(-(E_i - E_0)/(k T_vib)) (Eq. accept-quant; proposal range read as
 * inclusive of the ground state). Stream: pair = slot, cell, step = 0xFFFFFFFE. */
int orc_init_thermal(orc_ctx *o, const uint32_t *counts, const double *t_trans, const double *t_vib) {
  if (!o || !o->finalized) return E_STATE;
  uint32_t mm = o->max_modes;
  for (uint32_t c = 0; c < o->n_cells; ++c) {
    uint32_t n = 0;
    for (uint32_t s = 0; s < o->n_species; ++s) n += counts[(size_t)c * o->n_species + s];
    uint32_t cap = default_capacity(o, n);
    if (n > cap) return E_CAPACITY;
    if (!(t_trans[c] >= 0.0) || !(t_vib[c] >= 0.0)) return E_INVAL;
    int rc = alloc_cell(o, &o->cells[c], cap);
    if (rc) return rc;
    cell_t *C = &o->cells[c];
    memset(C->ctr, 0, sizeof(C->ctr));
    uint32_t slot = 0;
    for (uint32_t s = 0; s < o->n_species; ++s) {
      const species_t *S = &o->sp[s];
      double sigma = sqrt((K_BOLTZ * t_trans[c]) / S->mass);
      for (uint32_t k = 0; k < counts[(size_t)c * o->n_species + s]; ++k) {
        stream st;
        stream_open(&st, o->seed, slot, c, 0xFFFFFFFEu);
        double n1, n2, n3, n4;
        polar_normals(&st, &n1, &n2);
        polar_normals(&st, &n3, &n4);
        C->vx[slot] = sigma * n1;
        C->vy[slot] = sigma * n2;
        C->vz[slot] = sigma * n3;
        C->sp[slot] = (uint8_t)s;
        sample_internal(S, &st, t_vib[c], t_trans[c], C->lvl + (size_t)slot * mm, mm, &C->rot[slot]);
        if (o->spatial) {
          /* uniform in the cell: x = (i_x + u) L_x / n_x per axis */
          uint32_t ix = c % o->nx, iy = (c / o->nx) % o->ny, iz = c / (o->nx * o->ny);
          C->px[slot] = ((double)ix + uniform(&st)) * (o->len[0] / (double)o->nx);
          C->py[slot] = ((double)iy + uniform(&st)) * (o->len[1] / (double)o->ny);
          C->pz[slot] = ((double)iz + uniform(&st)) * (o->len[2] / (double)o->nz);
        }
        slot += 1;
      }
    }
    C->n = n;
    init_sgmax(o, C);
    init_sums(o, C);
  }
  o->step = 0;
  o->loaded = 1;
  reset_inflow(o);
  return E_OK;
}

/* ------------------------------------------------------------------ */
/* Vibrational relaxation (Sec. "Implementation of the polyatomic HCAO   */
/* model"): joint proposal + Larsen-Borgnakke acceptance, and the        */
/* single-mode (Gibbs sweep) form of the same conditional target.        */
/* ------------------------------------------------------------------ */

/* proposal range for mode m given the energy e available to the mode */
static uint32_t mode_top(const species_t *s, uint32_t m, double e) {
  if (m < s->n_bend) {
    /* i_max = floor(E/(k Theta) - 1/2) + 1 levels, i = floor(r i_max) in [0, i_max-1] */
    double fi = floor(e / s->kt[m] - 0.5);
    if (fi < 0.0) fi = 0.0;
    if (fi > 65535.0) fi = 65535.0;
    return (uint32_t)fi; /* inclusive top index */
  }
  /* highest stretch level strictly below the available energy, capped at i_diss */
  uint32_t top = 0;
  while (top < s->idiss[m] && s->lev[m][top + 1] < e) top += 1;
  return top;
}

static uint32_t propose(const species_t *s, uint32_t m, double e, double u) {
  uint32_t top = mode_top(s, m, e);
  double span = (double)top + 1.0;
  uint32_t i = (uint32_t)floor(u * span);
  if (i > top) i = top;
  return i;
}

/* Gibbs-sweep proposal for one mode (our sampler): the target
 * over levels 0..top is proportional to t_i = ((E_c - E_i) / den)^q with
 * den = E_c - E_0. Since (1 - x)^q <= 1 - q x for q in (0, 1], and a
 * concave level sequence has E_i - E_0 >= i (E_top - E_0) / top, t_i is
 * bounded by the linear envelope w_i = 1 - c i, c = q (E_top - E_0) /
 * (top den); the level is drawn from w_i and accepted with probability
 * t_i / w_i. The draw inverts the discrete CDF: with K = i + 1 the CDF is
 * G(K) = h K - (c/2) K^2, h = 1 + c/2, so i = floor(K*) with G(K*) = u G(top+1),
 * K* = 2 s / (h + sqrt(h^2 - 2 c s)). c = 0 (top = 0, or levels that are not
 * concave) is the uniform proposal floor(u (top + 1)). */
static double gibbs_slope(const species_t *s, uint32_t m, uint32_t top, double den, double q) {
  if (top == 0 || !s->concave[m]) return 0.0;
  return (q * (mode_energy(s, m, top) - mode_energy(s, m, 0))) / ((double)top * den);
}

static uint32_t propose_linear(uint32_t top, double c, double u) {
  double z = ((double)top + 1.0) * (1.0 - (0.5 * c) * (double)top);
  double h = 1.0 + 0.5 * c;
  double sv = u * z;
  double k = (2.0 * sv) / (h + sqrt(h * h - (2.0 * c) * sv));
  double fi = floor(k);
  uint32_t i = fi > (double)top ? top : (uint32_t)fi;
  return i;
}

uint32_t orc_gibbs_propose(uint32_t top, double c, double u) { return propose_linear(top, c, u); }

/* Exact sampler of the joint target (our design): the target of
 * the joint proposal, P(i) proportional to (E' - S(i))^q over S(i) < E' with
 * e_m(i) = E_m(i) - E_m(0), S = sum_m e_m(i_m) and E' = E_coll - ZPE, drawn by
 * rejection from a product of per-mode Boltzmann distributions at one inverse
 * temperature beta. With the proposal weight exp(-beta S), target / proposal
 * is (E' - S)^q exp(beta S); over S in [0, E') it peaks at S = E' - q / beta
 * (beta E' >= q), so the acceptance probability is
 * (y e^(1 - y))^q = exp(q (ln y + 1 - y)) with y = beta (E' - S) / q.
 * Any beta gives the target exactly; it sets only the acceptance rate, which
 * is highest where the proposal's mean energy plus q / beta equals E'.
 *
 * beta is looked up by E': the bin b = (bit pattern of E') >> 48 (1/16 of an
 * octave), clamped to [2^-90, 2^-49) J, holds beta_j of the grid
 * beta_j = (1 + (j mod 16) / 16) 2^(40 + j div 16), j in [0, 960): the smallest
 * j, by bisection, with G(beta_j) + q / beta_j <= E'_b, where E'_b is the
 * bin's midpoint and G the proposal's mean energy over the modes' full level
 * sets (bends: k Theta / expm1(beta k Theta); stretches: the Boltzmann mean of
 * e_i over 0..i_diss, i ascending). beta is raised to q / E' if below. */
#define EXACT_BIN_LO 14928u  /* bits(2^-90) >> 48 */
#define EXACT_BIN_HI 15583u  /* last bin below 2^-49 */
#define EXACT_NBETA 960u

static double exact_beta_grid(uint32_t j) { return ldexp(1.0 + (double)(j & 15u) / 16.0, (int)(j >> 4) + 40); }

static double exact_mean_energy(const species_t *s, double beta) {
  double g = 0.0;
  for (uint32_t m = 0; m < s->n_modes; ++m) {
    if (m < s->n_bend) {
      g = g + s->kt[m] / expm1(beta * s->kt[m]);
    } else {
      double num = 0.0, den = 0.0;
      for (uint32_t i = 0; i <= s->idiss[m]; ++i) {
        double e = s->lev[m][i] - s->lev[m][0];
        double w = exp(-(beta * e));
        num = num + e * w;
        den = den + w;
      }
      g = g + num / den;
    }
  }
  return g;
}

static uint32_t exact_bin(double ep) {
  uint64_t b;
  memcpy(&b, &ep, 8);
  uint32_t k = (uint32_t)(b >> 48);
  if (k < EXACT_BIN_LO) k = EXACT_BIN_LO;
  if (k > EXACT_BIN_HI) k = EXACT_BIN_HI;
  return k;
}

static double exact_bin_beta(const species_t *s, double q, uint32_t bin) {
  double ec = from_bits(((uint64_t)bin << 48) | ((uint64_t)1 << 47));
  uint32_t lo = 0, hi = EXACT_NBETA - 1;
  while (lo < hi) {
    uint32_t mid = (lo + hi) >> 1;
    double bm = exact_beta_grid(mid);
    if (exact_mean_energy(s, bm) + q / bm <= ec)
      hi = mid;
    else
      lo = mid + 1;
  }
  return exact_beta_grid(lo);
}

double orc_exact_beta(orc_ctx *o, uint32_t species, double q, double ep) {
  if (!o || species >= o->n_species || !(ep > 0.0)) return -1.0;
  double beta = exact_bin_beta(&o->sp[species], q, exact_bin(ep));
  if (beta * ep < q) beta = q / ep;
  return beta;
}

/* slope of the geometric proposal of mode m on 0..top: k Theta for bends;
 * for stretches the chord e(top) / top (a lower bound of e(i) / i when the
 * spacings never grow), else the minimum of e(i) / i */
static double exact_slope(const species_t *s, uint32_t m, uint32_t top) {
  if (m < s->n_bend) return s->kt[m];
  double e0 = s->lev[m][0];
  if (s->concave[m]) return (s->lev[m][top] - e0) / (double)top;
  double sl = s->lev[m][1] - e0;
  for (uint32_t i = 2; i <= top; ++i) {
    double v = (s->lev[m][i] - e0) / (double)i;
    if (v < sl) sl = v;
  }
  return sl;
}

static uint64_t relax_exact(const species_t *s, uint16_t *lvl, double *e_tr, double q, stream *st,
                            int *capped) {
  double e_coll = *e_tr + vib_energy(s, lvl);
  double ep = e_coll - s->zpe;
  if (!(ep > 0.0)) return 0;
  double beta = exact_bin_beta(s, q, exact_bin(ep));
  if (beta * ep < q) beta = q / ep;
  uint32_t top[ORC_MAX_MODES];
  double c[ORC_MAX_MODES], sl[ORC_MAX_MODES];
  for (uint32_t m = 0; m < s->n_modes; ++m) {
    top[m] = mode_top(s, m, ep + mode_energy(s, m, 0));
    sl[m] = top[m] > 0 ? exact_slope(s, m, top[m]) : 0.0;
    c[m] = beta * sl[m];
  }
  uint64_t trials = 0;
  uint16_t cand[ORC_MAX_MODES];
  for (;;) {
    double sum = 0.0;
    for (uint32_t m = 0; m < s->n_modes && !*capped; ++m) {
      cand[m] = 0;
      if (top[m] == 0) continue;
      for (;;) {
        trials += 1;
        if (trials >= ORC_MAX_TRIALS) {
          *capped = 1;
          break;
        }
        double u = uniform(st);
        double x = -orc_detlog(1.0 - u) / c[m];
        if (!(x < (double)top[m] + 1.0)) continue; /* beyond the top level: redraw */
        uint32_t i = (uint32_t)floor(x);
        if (m >= s->n_bend && i > 0) {
          /* stretch: keep with probability exp(-beta (e(i) - slope i)) */
          double d = (mode_energy(s, m, i) - mode_energy(s, m, 0)) - sl[m] * (double)i;
          if (d > 0.0) {
            double u2 = uniform(st);
            if (!(u2 < orc_detexp(-(beta * d)))) continue;
          }
        }
        cand[m] = (uint16_t)i;
        break;
      }
    }
    if (*capped) break;
    trials += 1;
    for (uint32_t m = 0; m < s->n_modes; ++m) sum = sum + (mode_energy(s, m, cand[m]) - mode_energy(s, m, 0));
    if (sum < ep) {
      double y = (beta * (ep - sum)) / q;
      double ua = uniform(st);
      if (ua < orc_detexp(q * ((orc_detlog(y) + 1.0) - y))) {
        for (uint32_t m = 0; m < s->n_modes; ++m) lvl[m] = cand[m];
        double ev = 0.0;
        for (uint32_t m = 0; m < s->n_modes; ++m) ev = ev + mode_energy(s, m, cand[m]);
        *e_tr = e_coll - ev;
        break;
      }
    }
    if (trials >= ORC_MAX_TRIALS) {
      *capped = 1;
      break;
    }
  }
  return trials;
}

/* Relaxes one molecule; *e_tr is the translational energy of the pair on
 * entry and on exit. Returns the number of trials. */
static uint64_t relax(const orc_ctx *o, const species_t *s, uint16_t *lvl, double *e_tr, double q,
                      stream *st, int *capped) {
  uint64_t trials = 0;
  *capped = 0;
  if (s->sampler == ORC_SAMPLER_EXACT) return relax_exact(s, lvl, e_tr, q, st, capped);
  if (s->sampler == ORC_SAMPLER_JOINT) {
    double e_coll = *e_tr + vib_energy(s, lvl);
    double denom = e_coll - s->zpe;
    if (!(denom > 0.0)) return 0;
    uint16_t cand[ORC_MAX_MODES];
    for (;;) {
      trials += 1;
      double sum = 0.0;
      for (uint32_t m = 0; m < s->n_modes; ++m) {
        double u = uniform(st);
        cand[m] = (uint16_t)propose(s, m, e_coll, u);
        sum = sum + mode_energy(s, m, cand[m]);
      }
      double ua = uniform(st);
      int accept = 0;
      if (sum < e_coll) accept = ua < orc_detpow((e_coll - sum) / denom, q);
      if (accept) {
        for (uint32_t m = 0; m < s->n_modes; ++m) lvl[m] = cand[m];
        *e_tr = e_coll - sum;
        break;
      }
      if (trials >= ORC_MAX_TRIALS) {
        *capped = 1;
        break;
      }
    }
    (void)o;
    return trials;
  }
  /* Gibbs sweep: each mode in turn takes the conditional of the joint target */
  double et = *e_tr;
  for (uint32_t m = 0; m < s->n_modes; ++m) {
    double ec = et + mode_energy(s, m, lvl[m]);
    double e0 = mode_energy(s, m, 0);
    double den = ec - e0;
    if (!(den > 0.0)) continue;
    uint32_t top = mode_top(s, m, ec);
    double c = gibbs_slope(s, m, top, den, q);
    for (;;) {
      trials += 1;
      double u = uniform(st);
      uint32_t i = propose_linear(top, c, u);
      double ei = mode_energy(s, m, i);
      double ua = uniform(st);
      int accept = 0;
      if (ei < ec) accept = ua * (1.0 - c * (double)i) < orc_detpow((ec - ei) / den, q);
      if (accept) {
        lvl[m] = (uint16_t)i;
        et = ec - ei;
        break;
      }
      if (trials >= ORC_MAX_TRIALS) {
        *capped = 1;
        break;
      }
    }
    if (*capped) break;
  }
  *e_tr = et;
  return trials;
}

/* ------------------------------------------------------------------ */
/* VHS isotropic scattering                                              */
/* ------------------------------------------------------------------ */
static void unit_vector(stream *st, double n[3]) {
  double x, y, s;
  for (;;) {
    x = 2.0 * uniform(st) - 1.0;
    y = 2.0 * uniform(st) - 1.0;
    s = x * x + y * y;
    if (s < 1.0) break;
  }
  double f = 2.0 * sqrt(1.0 - s);
  n[0] = x * f;
  n[1] = y * f;
  n[2] = 1.0 - 2.0 * s;
}

/* Dissociation into three bodies: share beta of the translational energy
 * that goes to the B-C relative motion. Two relative motions of three
 * translational degrees of freedom each give the density proportional to
 * sqrt(beta (1 - beta)) on (0, 1), a Beta(3/2, 3/2) law; drawn by rejection
 * from the uniform under its maximum 1/2. */
static double three_body_share(stream *st) {
  for (;;) {
    double u1 = uniform(st), u2 = uniform(st);
    if (u2 * 0.5 < sqrt(u1 * (1.0 - u1))) return u1;
  }
}

/* n draws of the scattering direction and of the three-body share, draw i
 * from the stream (seed; pair i, cell 0, step 0) */
void orc_draw_unit_vectors(uint64_t seed, uint32_t n, double *out) {
  for (uint32_t i = 0; i < n; ++i) {
    stream st;
    stream_open(&st, seed, i, 0, 0);
    unit_vector(&st, out + 3 * (size_t)i);
  }
}

void orc_draw_three_body_shares(uint64_t seed, uint32_t n, double *out) {
  for (uint32_t i = 0; i < n; ++i) {
    stream st;
    stream_open(&st, seed, i, 0, 0);
    out[i] = three_body_share(&st);
  }
}

/* Places two bodies (pair table p) about the centre-of-mass velocity vcm
 * with relative speed sqrt(2 E / m_r) along a random direction. */
static void split(const pair_t *p, const double vcm[3], double e, stream *st, double va[3], double vb[3]) {
  double g = sqrt((2.0 * e) / p->mr);
  double n[3];
  unit_vector(st, n);
  double ga = p->wa * g, gb = p->wb * g;
  for (int k = 0; k < 3; ++k) {
    va[k] = vcm[k] + ga * n[k];
    vb[k] = vcm[k] - gb * n[k];
  }
}

static void com(const pair_t *p, const double va[3], const double vb[3], double out[3]) {
  for (int k = 0; k < 3; ++k) out[k] = (p->m_a * va[k] + p->m_b * vb[k]) / p->msum;
}

/* ------------------------------------------------------------------ */
/* One accepted collision                                                */
/* ------------------------------------------------------------------ */
typedef struct {
  double v[2][3];
  uint8_t sp[2];
  uint16_t lvl[2][ORC_MAX_MODES];
  double rot[2];
  double pos[2][3];
  int dead[2];
  int has_m;   /* a third body is available for recombination */
  int m_moved; /* the third body took part (recombination) */
  uint8_t sp_m;
  double v_m[3];
  double t_cell, n_cell;
} pair_state;

typedef struct {
  int born;
  uint8_t sp;
  double v[3];
  uint16_t lvl[ORC_MAX_MODES];
  double rot;
  double pos[3]; /* spatial mode: the dissociating molecule's position */
} newborn;

/* Rotational Larsen-Borgnakke share (our rotor model): the fraction f of the
 * pooled energy E_tr + E_rot that the rotor keeps has density proportional to
 * f^(zeta/2 - 1) (1 - f)^q, q = 3/2 - omega the exponent of the vibrational
 * sampler. zeta = 2: inversion, f = 1 - (1 - u)^(1/(q+1)). zeta = 3: rejection
 * from the uniform, accepted with (f/f*)^(1/2) ((1 - f)/(1 - f*))^q, f* = 1/(1 + 2q)
 * the mode. */
static double rot_fraction(uint32_t zeta, double q, stream *st) {
  if (zeta == 2) return 1.0 - orc_detpow(1.0 - uniform(st), 1.0 / (q + 1.0));
  double fs = 1.0 / (1.0 + 2.0 * q);
  for (;;) {
    double f = uniform(st), u2 = uniform(st);
    if (u2 < orc_detpow(f / fs, 0.5) * orc_detpow((1.0 - f) / (1.0 - fs), q)) return f;
  }
}

typedef struct {
  int kind, rx, a_side, mode;
  double eex;
} channel;

#define MAX_CHANNELS 64

/* Reaction decision, application, or relaxation + scattering for one
 * accepted pair. Returns the reaction id or -1. ctr may be NULL. */
static int collide(const orc_ctx *o, pair_state *ps, double g2, stream *st, uint64_t *ctr, newborn *nb) {
  const pair_t *pp = &o->pr[ps->sp[0]][ps->sp[1]];
  double e_tr = pp->hm * g2;
  double evib[2];
  for (int x = 0; x < 2; ++x) evib[x] = vib_energy(&o->sp[ps->sp[x]], ps->lvl[x]);
  nb->born = 0;

  /* --- recombination first: B + C (+M) -> A (+M) --- */
  for (uint32_t r = 0; r < o->n_reactions; ++r) {
    const reaction_t *R = &o->rx[r];
    if (R->kind != ORC_RX_RECOMBINATION) continue;
    int side_b;
    if (ps->sp[0] == R->a && ps->sp[1] == R->b)
      side_b = 0;
    else if (ps->sp[1] == R->a && ps->sp[0] == R->b)
      side_b = 1;
    else
      continue;
    double u = uniform(st);
    if (!ps->has_m) {
      if (ctr) ctr[ORC_CTR_SUPPRESSED] += 1;
      continue;
    }
    double prob = rec_lookup(o, R, ps->sp_m, ps->t_cell) * ps->n_cell;
    if (prob > 1.0) prob = 1.0;
    if (!(u < prob)) continue;
    int b = side_b, c = 1 - side_b;
    const species_t *A = &o->sp[R->c];
    const pair_t *pbc = &o->pr[R->a][R->b];
    double vbc[3];
    com(pbc, ps->v[b], ps->v[c], vbc);
    double gx = vbc[0] - ps->v_m[0], gy = vbc[1] - ps->v_m[1], gz = vbc[2] - ps->v_m[2];
    const pair_t *pam = &o->pr[R->c][ps->sp_m];
    double e_am = pam->hm * ((gx * gx + gy * gy) + gz * gz);
    double pool = (((e_am + e_tr) + evib[b]) + evib[c]) - R->dh;
    /* rotation of B and C: kept by A's rotor, else pooled */
    double rsum = ps->rot[b] + ps->rot[c];
    if (A->zeta_rot == 0) pool = pool + rsum;
    double et = pool - A->zpe;
    if (!(et > 0.0)) {
      if (ctr) ctr[ORC_CTR_SUPPRESSED] += 1;
      continue;
    }
    uint16_t la[ORC_MAX_MODES] = {0};
    int capped = 0;
    uint64_t t = relax(o, A, la, &et, pam->q, st, &capped);
    double vcm[3], va[3], vm[3];
    com(pam, vbc, ps->v_m, vcm);
    split(pam, vcm, et, st, va, vm);
    memcpy(ps->v[b], va, sizeof(va));
    memcpy(ps->v_m, vm, sizeof(vm));
    ps->m_moved = 1;
    ps->sp[b] = (uint8_t)R->c;
    memcpy(ps->lvl[b], la, sizeof(la));
    ps->rot[b] = A->zeta_rot > 0 ? rsum : 0.0;
    ps->rot[c] = 0.0;
    ps->dead[c] = 1;
    if (ctr) {
      ctr[ORC_CTR_TRIALS] += t;
      ctr[ORC_CTR_CAPPED] += (uint64_t)capped;
      ctr[ORC_CTR_DEATHS] += 1;
      ctr[ORC_CTR_REACTION0 + r] += 1;
    }
    return (int)r;
  }

  /* --- reaction decision: dissociation then exchange channels, canonical order --- */
  channel ch[MAX_CHANNELS];
  int nch = 0;
  for (int side = 0; side < 2; ++side) {
    int A = ps->sp[side];
    for (uint32_t r = 0; r < o->n_reactions; ++r) {
      const reaction_t *R = &o->rx[r];
      if (R->kind != ORC_RX_DISSOCIATION || R->a != A) continue;
      const species_t *SA = &o->sp[A];
      for (uint32_t j = 0; j < SA->n_stretch; ++j) {
        if (!((R->mask >> j) & 1ULL)) continue;
        uint32_t m = SA->n_bend + j;
        /* Eq. Ecoll-diss (with rotation coupling): E_tr + gamma E_rot,A + E_vib,A
         * - sum of ZPE over A, B, C + E_A,j(0) */
        double grot = R->gamma_rot * ps->rot[side];
        double ecoll = (((e_tr + grot) + evib[side]) - R->zsum) + SA->lev[m][0];
        double eex = ecoll - SA->de[m];
        double pool = ((e_tr + grot) + evib[side]) - R->dh;
        double left = (pool - o->sp[R->c].zpe) - o->sp[R->d].zpe;
        if (eex > 0.0 && left > 0.0 && nch < MAX_CHANNELS) {
          ch[nch].kind = ORC_RX_DISSOCIATION;
          ch[nch].rx = (int)r;
          ch[nch].a_side = side;
          ch[nch].mode = (int)m;
          ch[nch].eex = eex;
          nch += 1;
        }
      }
    }
  }
  for (int side = 0; side < 2; ++side) {
    int A = ps->sp[side], B = ps->sp[1 - side];
    for (uint32_t r = 0; r < o->n_reactions; ++r) {
      const reaction_t *R = &o->rx[r];
      if (R->kind != ORC_RX_EXCHANGE || R->a != A || R->b != B) continue;
      double us = uniform(st);
      const species_t *SA = &o->sp[A];
      /* Eq. Ecoll-exch (with rotation coupling): E_tr + gamma E_rot,A + sum_j alpha_j E_vib,A,j */
      double grot = R->gamma_rot * ps->rot[side];
      double ecoll = e_tr + grot;
      for (uint32_t m = 0; m < SA->n_modes; ++m)
        ecoll = ecoll + R->alpha[m] * mode_energy(SA, m, ps->lvl[side][m]);
      double eex = ecoll - R->ea;
      double pool = (((e_tr + grot) + evib[side]) + evib[1 - side]) - R->dh;
      double left = (pool - o->sp[R->c].zpe) - o->sp[R->d].zpe;
      if (us < R->steric && eex > 0.0 && left > 0.0 && nch < MAX_CHANNELS) {
        ch[nch].kind = ORC_RX_EXCHANGE;
        ch[nch].rx = (int)r;
        ch[nch].a_side = side;
        ch[nch].mode = -1;
        ch[nch].eex = eex;
        nch += 1;
      }
    }
  }
  int pick = -1;
  if (nch == 1) {
    pick = 0;
  } else if (nch > 1) {
    /* one draw, channels weighted by their excess energy */
    double total = 0.0;
    for (int c = 0; c < nch; ++c) total = total + ch[c].eex;
    double target = uniform(st) * total;
    double cum = 0.0;
    pick = nch - 1;
    for (int c = 0; c < nch; ++c) {
      cum = cum + ch[c].eex;
      if (target < cum) {
        pick = c;
        break;
      }
    }
  }

  if (pick >= 0) {
    const reaction_t *R = &o->rx[ch[pick].rx];
    int a = ch[pick].a_side, b = 1 - a;
    if (R->kind == ORC_RX_DISSOCIATION) {
      /* A + M -> B + C + M: B takes A's slot, C is new. */
      int spA = ps->sp[a], spM = ps->sp[b];
      double grot = R->gamma_rot * ps->rot[a];
      double pool = ((e_tr + grot) + evib[a]) - R->dh;
      double et = (pool - o->sp[R->c].zpe) - o->sp[R->d].zpe;
      /* the rotation not coupled in stays with B's rotor, else is pooled */
      double keep = ps->rot[a] - grot;
      if (o->sp[R->c].zeta_rot == 0) {
        et = et + keep;
        keep = 0.0;
      }
      uint16_t lb[ORC_MAX_MODES] = {0}, lc[ORC_MAX_MODES] = {0};
      int capped = 0;
      uint64_t t = 0;
      if (o->sp[R->c].n_modes > 0) t += relax(o, &o->sp[R->c], lb, &et, o->pr[R->c][spM].q, st, &capped);
      if (o->sp[R->d].n_modes > 0) {
        int c2 = 0;
        t += relax(o, &o->sp[R->d], lc, &et, o->pr[R->d][spM].q, st, &c2);
        capped |= c2;
      }
      double beta = three_body_share(st);
      double ebc = beta * et;
      double exm = et - ebc;
      const pair_t *pam = &o->pr[spA][spM];
      double vcm[3], vbc[3], vm[3], vbn[3], vcn[3];
      com(pam, ps->v[a], ps->v[b], vcm);
      split(pam, vcm, exm, st, vbc, vm);
      split(&o->pr[R->c][R->d], vbc, ebc, st, vbn, vcn);
      for (int k = 0; k < 3; ++k) {
        ps->v[a][k] = vbn[k];
        ps->v[b][k] = vm[k];
        nb->v[k] = vcn[k];
      }
      ps->sp[a] = (uint8_t)R->c;
      memcpy(ps->lvl[a], lb, sizeof(lb));
      ps->rot[a] = keep;
      nb->born = 1;
      nb->sp = (uint8_t)R->d;
      memcpy(nb->lvl, lc, sizeof(lc));
      nb->rot = 0.0;
      for (int k = 0; k < 3; ++k) nb->pos[k] = ps->pos[a][k];
      if (ctr) {
        ctr[ORC_CTR_TRIALS] += t;
        ctr[ORC_CTR_CAPPED] += (uint64_t)capped;
        ctr[ORC_CTR_BIRTHS] += 1;
        ctr[ORC_CTR_REACTION0 + ch[pick].rx] += 1;
      }
    } else {
      /* A + B -> C + D: C takes A's slot, D takes B's slot. */
      int spA = ps->sp[a], spB = ps->sp[b];
      double grot = R->gamma_rot * ps->rot[a];
      double pool = (((e_tr + grot) + evib[a]) + evib[b]) - R->dh;
      double et = (pool - o->sp[R->c].zpe) - o->sp[R->d].zpe;
      /* A's uncoupled rotation goes to C's rotor, B's to D's; else pooled */
      double keep_c = ps->rot[a] - grot, keep_d = ps->rot[b];
      if (o->sp[R->c].zeta_rot == 0) {
        et = et + keep_c;
        keep_c = 0.0;
      }
      if (o->sp[R->d].zeta_rot == 0) {
        et = et + keep_d;
        keep_d = 0.0;
      }
      uint16_t lc[ORC_MAX_MODES] = {0}, ld[ORC_MAX_MODES] = {0};
      double qcd = o->pr[R->c][R->d].q;
      int capped = 0;
      uint64_t t = 0;
      if (o->sp[R->c].n_modes > 0) t += relax(o, &o->sp[R->c], lc, &et, qcd, st, &capped);
      if (o->sp[R->d].n_modes > 0) {
        int c2 = 0;
        t += relax(o, &o->sp[R->d], ld, &et, qcd, st, &c2);
        capped |= c2;
      }
      double vcm[3], vc[3], vd[3];
      com(&o->pr[spA][spB], ps->v[a], ps->v[b], vcm);
      split(&o->pr[R->c][R->d], vcm, et, st, vc, vd);
      memcpy(ps->v[a], vc, sizeof(vc));
      memcpy(ps->v[b], vd, sizeof(vd));
      ps->sp[a] = (uint8_t)R->c;
      ps->sp[b] = (uint8_t)R->d;
      memcpy(ps->lvl[a], lc, sizeof(lc));
      memcpy(ps->lvl[b], ld, sizeof(ld));
      ps->rot[a] = keep_c;
      ps->rot[b] = keep_d;
      if (ctr) {
        ctr[ORC_CTR_TRIALS] += t;
        ctr[ORC_CTR_CAPPED] += (uint64_t)capped;
        ctr[ORC_CTR_REACTION0 + ch[pick].rx] += 1;
      }
    }
    return ch[pick].rx;
  }

  /* --- no reaction: relax each molecule in turn, then scatter --- */
  for (int x = 0; x < 2; ++x) {
    const species_t *S = &o->sp[ps->sp[x]];
    if (S->n_modes == 0) continue;
    double u = uniform(st);
    if (!(u < S->p_vib)) continue;
    int capped = 0;
    uint64_t t = relax(o, S, ps->lvl[x], &e_tr, pp->q, st, &capped);
    if (ctr) {
      ctr[ORC_CTR_TRIALS] += t;
      ctr[ORC_CTR_RELAX] += 1;
      ctr[ORC_CTR_CAPPED] += (uint64_t)capped;
    }
  }
  /* rotational relaxation of each rotor in turn, after the vibrational one */
  for (int x = 0; x < 2; ++x) {
    const species_t *S = &o->sp[ps->sp[x]];
    if (S->zeta_rot == 0) continue;
    double u = uniform(st);
    if (!(u < S->p_rot)) continue;
    double ec = e_tr + ps->rot[x];
    double f = rot_fraction(S->zeta_rot, pp->q, st);
    ps->rot[x] = f * ec;
    e_tr = ec - ps->rot[x];
  }
  double vcm[3], va[3], vb[3];
  com(pp, ps->v[0], ps->v[1], vcm);
  split(pp, vcm, e_tr, st, va, vb);
  memcpy(ps->v[0], va, sizeof(va));
  memcpy(ps->v[1], vb, sizeof(vb));
  return -1;
}

/* ------------------------------------------------------------------ */
/* One time step of one cell                                             */
/* ------------------------------------------------------------------ */
static void load_pair(const cell_t *C, uint32_t mm, uint32_t p, uint32_t q, pair_state *ps) {
  uint32_t idx[2] = {p, q};
  memset(ps, 0, sizeof(*ps));
  for (int x = 0; x < 2; ++x) {
    uint32_t i = idx[x];
    ps->v[x][0] = C->vx[i];
    ps->v[x][1] = C->vy[i];
    ps->v[x][2] = C->vz[i];
    ps->sp[x] = C->sp[i];
    ps->rot[x] = C->rot[i];
    if (C->px) {
      ps->pos[x][0] = C->px[i];
      ps->pos[x][1] = C->py[i];
      ps->pos[x][2] = C->pz[i];
    }
    for (uint32_t m = 0; m < mm; ++m) ps->lvl[x][m] = C->lvl[(size_t)i * mm + m];
  }
}

static void store_pair(cell_t *C, uint32_t mm, uint32_t p, uint32_t q, const pair_state *ps) {
  uint32_t idx[2] = {p, q};
  for (int x = 0; x < 2; ++x) {
    uint32_t i = idx[x];
    C->vx[i] = ps->v[x][0];
    C->vy[i] = ps->v[x][1];
    C->vz[i] = ps->v[x][2];
    C->sp[i] = ps->dead[x] ? (uint8_t)255 : ps->sp[x];
    for (uint32_t m = 0; m < mm; ++m) C->lvl[(size_t)i * mm + m] = ps->lvl[x][m];
    C->rot[i] = ps->rot[x];
  }
}

/* Sums of m, m v_x, m v_y, m v_z and m |v|^2 over a cell's particles (m the
 * particle's mass). Summation order (fixed, so that every implementation
 * rounds alike): partial sum t (t = 0..63) takes the particles t, t + 64,
 * t + 128, ... in slot order; the 64 partial sums are then combined by a
 * halving tree (sum t adds sum t + s for s = 32, 16, ..., 1). */
static void cell_sums(const orc_ctx *o, const cell_t *C, double out[5]) {
  uint32_t n = C->n;
  double x[5][64];
  for (int t = 0; t < 64; ++t) {
    for (int q = 0; q < 5; ++q) x[q][t] = 0.0;
    for (uint32_t i = (uint32_t)t; i < n; i += 64) {
      double m = o->sp[C->sp[i]].mass;
      double vx = C->vx[i], vy = C->vy[i], vz = C->vz[i];
      x[0][t] = x[0][t] + m;
      x[1][t] = x[1][t] + m * vx;
      x[2][t] = x[2][t] + m * vy;
      x[3][t] = x[3][t] + m * vz;
      x[4][t] = x[4][t] + m * ((vx * vx + vy * vy) + vz * vz);
    }
  }
  for (int sft = 32; sft >= 1; sft >>= 1)
    for (int t = 0; t < sft; ++t)
      for (int q = 0; q < 5; ++q) x[q][t] = x[q][t] + x[q][t + sft];
  for (int q = 0; q < 5; ++q) out[q] = x[q][0];
}

/* The running sums start from the particles whenever a cell's particles are
 * placed (load, thermal initial state, every re-bin of the spatial mode) and
 * then follow each step's collisions (see step_cell). */
static void init_sums(const orc_ctx *o, cell_t *C) {
  if (o->has_recomb) cell_sums(o, C, C->tsum);
}

/* Translational temperature of a cell at step start from its running sums,
 * T = (sum m |v|^2 - |sum m v|^2 / sum m) / (3 k N): the sum of m |v - u|^2
 * about the mass-weighted mean velocity u over 3 k N (0 below two particles). */
static double cell_temperature(const orc_ctx *o, const cell_t *C) {
  (void)o;
  uint32_t n = C->n;
  if (n < 2) return 0.0;
  const double *s = C->tsum;
  double p2 = (s[1] * s[1] + s[2] * s[2]) + s[3] * s[3];
  return (s[4] - p2 / s[0]) / (3.0 * K_BOLTZ * (double)n);
}

/* adds one particle's five terms (m, m v, m |v|^2) to acc, in that order */
static void add_terms(double acc[5], double m, const double v[3]) {
  acc[0] = acc[0] + m;
  acc[1] = acc[1] + m * v[0];
  acc[2] = acc[2] + m * v[1];
  acc[3] = acc[3] + m * v[2];
  acc[4] = acc[4] + m * ((v[0] * v[0] + v[1] * v[1]) + v[2] * v[2]);
}

double orc_cell_temperature(const orc_ctx *o, uint32_t cell) {
  if (!o || cell >= o->n_cells) return -1.0;
  return cell_temperature(o, &o->cells[cell]);
}

int orc_cell_sums(const orc_ctx *o, uint32_t cell, int direct, double *out5) {
  if (!o || cell >= o->n_cells || !out5) return E_INVAL;
  if (direct)
    cell_sums(o, &o->cells[cell], out5);
  else
    memcpy(out5, o->cells[cell].tsum, 5 * sizeof(double));
  return E_OK;
}

static int step_cell(orc_ctx *o, uint32_t c, double dt) {
  cell_t *C = &o->cells[c];
  uint32_t mm = o->max_modes;
  uint32_t n = C->n;
  /* NTC: N_cand = floor(1/2 N (N-1) F_N (sigma g)_max dt / V + remainder) */
  double x = 0.5 * (double)n * (double)(n - (n > 0 ? 1 : 0)) * C->weight * C->sgmax * dt / C->volume + C->rem;
  double fl = floor(x);
  C->rem = x - fl;
  uint64_t ncand = (uint64_t)fl;
  if (ncand > n / 2) {
    C->ctr[ORC_CTR_SUPPRESSED] += ncand - n / 2;
    ncand = n / 2;
  }
  /* sixteen Feistel round keys: blocks 0..3 of the cell stream */
  uint32_t keys[16];
  for (uint32_t blk = 0; blk < 4; ++blk) {
    uint32_t ctr[4] = {blk, 0xFFFFFFFFu, c, o->step};
    orc_philox4x32_10((uint32_t)o->seed, (uint32_t)(o->seed >> 32), ctr, keys + 4 * blk);
  }
  newborn *nb = NULL;
  double *dsum = NULL;    /* recombination: each pair's change of the running sums */
  uint8_t *moved = NULL;  /* the pair collided */
  if (ncand > 0) {
    nb = (newborn *)calloc(ncand, sizeof(newborn));
    dsum = (double *)calloc((size_t)ncand * 5, sizeof(double));
    moved = (uint8_t *)calloc(ncand, 1);
    if (!nb || !dsum || !moved) {
      free(nb);
      free(dsum);
      free(moved);
      return E_NOMEM;
    }
  }
  double t_cell = o->has_recomb ? cell_temperature(o, C) : 0.0;
  double n_cell = (double)n * C->weight / C->volume;
  double sg_seen = 0.0;
  for (uint32_t k = 0; k < ncand; ++k) {
    uint32_t p = orc_feistel_index(n, keys, 2 * k);
    uint32_t q = orc_feistel_index(n, keys, 2 * k + 1);
    stream st;
    stream_open(&st, o->seed, k, c, o->step);
    C->ctr[ORC_CTR_CANDIDATES] += 1;
    double dx = C->vx[p] - C->vx[q], dy = C->vy[p] - C->vy[q], dz = C->vz[p] - C->vz[q];
    double g2 = (dx * dx + dy * dy) + dz * dz;
    const pair_t *pp = &o->pr[C->sp[p]][C->sp[q]];
    double sg = (g2 > 0.0) ? pp->csg * orc_detpow(g2, pp->esg) : 0.0;
    if (sg > sg_seen) sg_seen = sg;
    double ua = uniform(&st);
    if (!(ua < sg / C->sgmax)) continue;
    C->ctr[ORC_CTR_COLLISIONS] += 1;
    pair_state ps;
    load_pair(C, mm, p, q, &ps);
    ps.m_moved = 0;
    /* third body of pair k: the particle at permutation index 2 N_cand + k */
    uint32_t mslot = 0;
    if (2 * ncand + k < n) {
      mslot = orc_feistel_index(n, keys, (uint32_t)(2 * ncand + k));
      ps.has_m = 1;
      ps.sp_m = C->sp[mslot];
      ps.v_m[0] = C->vx[mslot];
      ps.v_m[1] = C->vy[mslot];
      ps.v_m[2] = C->vz[mslot];
    }
    ps.t_cell = t_cell;
    ps.n_cell = n_cell;
    double before[5] = {0.0, 0.0, 0.0, 0.0, 0.0}, vm_before[3] = {ps.v_m[0], ps.v_m[1], ps.v_m[2]};
    uint8_t sp_before[2] = {ps.sp[0], ps.sp[1]};
    double v_before[2][3];
    memcpy(v_before, ps.v, sizeof(v_before));
    collide(o, &ps, g2, &st, C->ctr, &nb[k]);
    if (o->has_recomb) {
      /* this pair's change of the running sums: its particles after the
       * collision (p, q, the third body if it took part, the newborn) minus
       * before (p, q, the third body if it took part) */
      add_terms(before, o->sp[sp_before[0]].mass, v_before[0]);
      add_terms(before, o->sp[sp_before[1]].mass, v_before[1]);
      if (ps.m_moved) add_terms(before, o->sp[ps.sp_m].mass, vm_before);
      double after[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
      if (!ps.dead[0]) add_terms(after, o->sp[ps.sp[0]].mass, ps.v[0]);
      if (!ps.dead[1]) add_terms(after, o->sp[ps.sp[1]].mass, ps.v[1]);
      if (ps.m_moved) add_terms(after, o->sp[ps.sp_m].mass, ps.v_m);
      if (nb[k].born) add_terms(after, o->sp[nb[k].sp].mass, nb[k].v);
      for (int qq = 0; qq < 5; ++qq) dsum[(size_t)k * 5 + qq] = after[qq] - before[qq];
      moved[k] = 1;
    }
    store_pair(C, mm, p, q, &ps);
    if (ps.has_m) {
      C->vx[mslot] = ps.v_m[0];
      C->vy[mslot] = ps.v_m[1];
      C->vz[mslot] = ps.v_m[2];
    }
  }
  /* deaths removed (survivors keep their order), births appended in pair order */
  uint32_t alive = 0;
  for (uint32_t i = 0; i < n; ++i) {
    if (C->sp[i] == 255) continue;
    if (alive != i) {
      C->vx[alive] = C->vx[i];
      C->vy[alive] = C->vy[i];
      C->vz[alive] = C->vz[i];
      C->sp[alive] = C->sp[i];
      C->rot[alive] = C->rot[i];
      if (C->px) {
        C->px[alive] = C->px[i];
        C->py[alive] = C->py[i];
        C->pz[alive] = C->pz[i];
      }
      for (uint32_t m = 0; m < mm; ++m) C->lvl[(size_t)alive * mm + m] = C->lvl[(size_t)i * mm + m];
    }
    ++alive;
  }
  C->n = alive;
  uint32_t births = 0;
  for (uint32_t k = 0; k < ncand; ++k) births += (uint32_t)nb[k].born;
  if (alive + births > C->cap) {
    free(nb);
    free(dsum);
    free(moved);
    return E_CAPACITY;
  }
  for (uint32_t k = 0; k < ncand; ++k) {
    if (!nb[k].born) continue;
    uint32_t j = C->n++;
    C->vx[j] = nb[k].v[0];
    C->vy[j] = nb[k].v[1];
    C->vz[j] = nb[k].v[2];
    C->sp[j] = nb[k].sp;
    C->rot[j] = nb[k].rot;
    if (C->px) {
      C->px[j] = nb[k].pos[0];
      C->py[j] = nb[k].pos[1];
      C->pz[j] = nb[k].pos[2];
    }
    for (uint32_t m = 0; m < mm; ++m) C->lvl[(size_t)j * mm + m] = nb[k].lvl[m];
  }
  if (o->has_recomb) {
    /* running sums: the pairs' changes over chunks of 64 consecutive
     * candidates (left to right), each chunk reduced by a halving tree; a
     * candidate that did not collide contributes 0 */
    double d[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (uint64_t k0 = 0; k0 < ncand; k0 += 64) {
      double x[5][64];
      for (int t = 0; t < 64; ++t)
        for (int qq = 0; qq < 5; ++qq)
          x[qq][t] = (k0 + t < ncand && moved[k0 + t]) ? dsum[(size_t)(k0 + t) * 5 + qq] : 0.0;
      for (int sft = 32; sft >= 1; sft >>= 1)
        for (int t = 0; t < sft; ++t)
          for (int qq = 0; qq < 5; ++qq) x[qq][t] = x[qq][t] + x[qq][t + sft];
      for (int qq = 0; qq < 5; ++qq) d[qq] = d[qq] + x[qq][0];
    }
    for (int qq = 0; qq < 5; ++qq) C->tsum[qq] = C->tsum[qq] + d[qq];
  }
  free(nb);
  free(dsum);
  free(moved);
  if (sg_seen > C->sgmax) C->sgmax = sg_seen;
  return E_OK;
}

/* an inserted particle, held until the re-bin */
typedef struct {
  double v[3], p[3], rot;
  uint16_t lvl[ORC_MAX_MODES];
  uint8_t sp;
  uint32_t cell; /* UINT32_MAX: left again during its partial flight */
} inflow_t;

/* The particles the open faces admit this step (faces in order, face cells
 * in order, species in order). Particle i of species s at face cell j of
 * face f draws from the stream pair = (s << 24) | i, cell = n_cells + the
 * face cell's index over all six faces, step = the step: the normal speed
 * from the flux-weighted Maxwellian, v_n = sigma sqrt(-2 ln(1 - u)); the two
 * tangential components, sigma times a polar normal pair; the fraction tau
 * of the step it flies; its place on the face cell, uniform on each
 * tangential axis; then levels at t_vib and rotational energy at t_trans as
 * the thermal initial state draws them. It enters at the face and moves
 * over tau dt with the box's boundaries. */
static int make_inflow(orc_ctx *o, double dt, inflow_t **out, uint64_t *n_out) {
  uint32_t mm = o->max_modes ? o->max_modes : 1;
  uint64_t n = 0, cap = 0;
  inflow_t *list = NULL;
  uint32_t base = 0;
  for (uint32_t f = 0; f < 6; ++f) {
    int a, b;
    uint32_t size;
    face_axes(o, f, &a, &b, &size);
    if (!((o->open_faces >> f) & 1u)) {
      base += size;
      continue;
    }
    int k = (int)(f >> 1), side = (int)(f & 1u);
    uint32_t na = axis_cells(o, a), nb = axis_cells(o, b), nk = axis_cells(o, k);
    double da = o->len[a] / (double)na, db = o->len[b] / (double)nb;
    double area = da * db;
    for (uint32_t j = 0; j < size; ++j) {
      uint32_t idx[3];
      idx[k] = side ? nk - 1 : 0;
      idx[a] = j % na;
      idx[b] = j / na;
      uint32_t c = idx[0] + o->nx * (idx[1] + o->ny * idx[2]);
      double weight = o->cells[c].weight;
      for (uint32_t s = 0; s < o->n_species; ++s) {
        double *rem = &o->in_rem[(size_t)(base + j) * o->n_species + s];
        double x = ((o->in_flux[s] * area) * dt) / weight + *rem;
        double fl = floor(x);
        if (!(fl < 16777216.0)) {
          free(list);
          return E_INVAL;
        }
        uint32_t cnt = (uint32_t)fl;
        *rem = x - fl;
        const species_t *S = &o->sp[s];
        double sigma = sqrt((K_BOLTZ * o->in_t) / S->mass);
        for (uint32_t i = 0; i < cnt; ++i) {
          if (n == cap) {
            cap = cap ? 2 * cap : 1024;
            inflow_t *nl = (inflow_t *)realloc(list, cap * sizeof(inflow_t));
            if (!nl) {
              free(list);
              return E_NOMEM;
            }
            list = nl;
          }
          inflow_t *P = &list[n++];
          stream st;
          stream_open(&st, o->seed, (s << 24) | i, o->n_cells + base + j, o->step);
          double vn = sigma * sqrt(-2.0 * orc_detlog(1.0 - uniform(&st)));
          double n1, n2;
          polar_normals(&st, &n1, &n2);
          double tau = uniform(&st);
          double ua = uniform(&st);
          double ub = uniform(&st);
          P->p[k] = side ? o->len[k] : 0.0;
          P->v[k] = side ? -vn : vn;
          P->p[a] = ((double)idx[a] + ua) * da;
          P->p[b] = ((double)idx[b] + ub) * db;
          P->v[a] = sigma * n1;
          P->v[b] = sigma * n2;
          P->sp = (uint8_t)s;
          sample_internal(S, &st, o->in_tv, o->in_t, P->lvl, mm, &P->rot);
          if (move_particle(o, &P->p[0], &P->p[1], &P->p[2], &P->v[0], &P->v[1], &P->v[2], tau * dt))
            P->cell = UINT32_MAX;
          else
            P->cell = cell_of(o, P->p[0], P->p[1], P->p[2]);
        }
      }
    }
    base += size;
  }
  *out = list;
  *n_out = n;
  return E_OK;
}

/* Spatial mode: every particle moves over dt (cells in order, particles in
 * slot order; one that crosses an open face leaves), the open faces admit
 * their particles, then all are re-binned by their new cell: within each
 * new cell the particles already in the box keep their order and the
 * admitted ones follow in the order they were made. */
static int move_and_rebin(orc_ctx *o, double dt) {
  uint32_t mm = o->max_modes ? o->max_modes : 1;
  uint32_t *newn = (uint32_t *)calloc(o->n_cells, sizeof(uint32_t));
  uint32_t **dest = (uint32_t **)calloc(o->n_cells, sizeof(uint32_t *));
  if (!newn || !dest) {
    free(newn);
    free(dest);
    return E_NOMEM;
  }
  int rc = E_OK;
  for (uint32_t c = 0; c < o->n_cells && !rc; ++c) {
    cell_t *C = &o->cells[c];
    dest[c] = (uint32_t *)malloc((C->n ? C->n : 1) * sizeof(uint32_t));
    if (!dest[c]) {
      rc = E_NOMEM;
      break;
    }
    for (uint32_t i = 0; i < C->n; ++i) {
      if (move_particle(o, &C->px[i], &C->py[i], &C->pz[i], &C->vx[i], &C->vy[i], &C->vz[i], dt)) {
        dest[c][i] = UINT32_MAX;
        o->flux_out += 1;
      } else {
        dest[c][i] = cell_of(o, C->px[i], C->py[i], C->pz[i]);
        newn[dest[c][i]] += 1;
      }
    }
  }
  inflow_t *ins = NULL;
  uint64_t n_ins = 0;
  if (!rc && o->open_faces) rc = make_inflow(o, dt, &ins, &n_ins);
  for (uint64_t i = 0; i < n_ins && !rc; ++i) {
    o->flux_in += 1;
    if (ins[i].cell == UINT32_MAX)
      o->flux_out += 1;
    else
      newn[ins[i].cell] += 1;
  }
  for (uint32_t c = 0; c < o->n_cells && !rc; ++c)
    if (newn[c] > o->cells[c].cap) rc = E_CAPACITY;
  cell_t *nc = NULL;
  if (!rc) {
    nc = (cell_t *)calloc(o->n_cells, sizeof(cell_t));
    if (!nc) rc = E_NOMEM;
  }
  for (uint32_t c = 0; c < o->n_cells && !rc; ++c) {
    rc = alloc_cell(o, &nc[c], o->cells[c].cap);
    nc[c].volume = o->cells[c].volume;
    nc[c].weight = o->cells[c].weight;
    nc[c].sgmax = o->cells[c].sgmax;
    nc[c].rem = o->cells[c].rem;
    memcpy(nc[c].ctr, o->cells[c].ctr, sizeof(nc[c].ctr));
  }
  for (uint32_t c = 0; c < o->n_cells && !rc; ++c) {
    cell_t *C = &o->cells[c];
    for (uint32_t i = 0; i < C->n; ++i) {
      if (dest[c][i] == UINT32_MAX) continue;
      cell_t *D = &nc[dest[c][i]];
      uint32_t j = D->n++;
      D->vx[j] = C->vx[i];
      D->vy[j] = C->vy[i];
      D->vz[j] = C->vz[i];
      D->sp[j] = C->sp[i];
      D->rot[j] = C->rot[i];
      D->px[j] = C->px[i];
      D->py[j] = C->py[i];
      D->pz[j] = C->pz[i];
      for (uint32_t m = 0; m < mm; ++m) D->lvl[(size_t)j * mm + m] = C->lvl[(size_t)i * mm + m];
    }
  }
  for (uint64_t i = 0; i < n_ins && !rc; ++i) {
    const inflow_t *P = &ins[i];
    if (P->cell == UINT32_MAX) continue;
    cell_t *D = &nc[P->cell];
    uint32_t j = D->n++;
    D->vx[j] = P->v[0];
    D->vy[j] = P->v[1];
    D->vz[j] = P->v[2];
    D->sp[j] = P->sp;
    D->rot[j] = P->rot;
    D->px[j] = P->p[0];
    D->py[j] = P->p[1];
    D->pz[j] = P->p[2];
    for (uint32_t m = 0; m < mm; ++m) D->lvl[(size_t)j * mm + m] = P->lvl[m];
  }
  if (nc) {
    for (uint32_t c = 0; c < o->n_cells; ++c) {
      if (!rc) {
        free_cell(&o->cells[c]);
        o->cells[c] = nc[c];
      } else {
        free_cell(&nc[c]);
      }
    }
  }
  free(nc);
  for (uint32_t c = 0; c < o->n_cells; ++c) free(dest[c]);
  free(dest);
  free(ins);
  free(newn);
  return rc;
}

int orc_set_threads(orc_ctx *o, int n) {
  if (!o || n < 0) return E_INVAL;
  o->threads = n;
  return E_OK;
}

int orc_step(orc_ctx *o, double dt, uint32_t n_steps) {
  if (!o || !o->loaded) return E_STATE;
  if (!(dt > 0.0)) return E_INVAL;
  for (uint32_t s = 0; s < n_steps; ++s) {
    if (o->spatial) {
      int rc = move_and_rebin(o, dt);
      if (rc) return rc;
      for (uint32_t c = 0; c < o->n_cells; ++c) init_sums(o, &o->cells[c]);
    }
    /* cells are independent (per-cell state, per-cell streams), so threads
     * over cells give the same result as one thread */
    int first = E_OK;
#pragma omp parallel for schedule(static) num_threads(o->threads > 0 ? o->threads : 1)
    for (uint32_t c = 0; c < o->n_cells; ++c) {
      int rc = step_cell(o, c, dt);
      if (rc) {
#pragma omp critical
        if (first == E_OK) first = rc;
      }
    }
    if (first != E_OK) return first;
    o->step += 1;
  }
  return E_OK;
}

/* ------------------------------------------------------------------ */
/* Queries                                                               */
/* ------------------------------------------------------------------ */
uint32_t orc_max_modes(const orc_ctx *o) { return o->max_modes; }
uint64_t orc_count(const orc_ctx *o, uint32_t cell) { return cell < o->n_cells ? o->cells[cell].n : 0; }
uint32_t orc_step_index(const orc_ctx *o) { return o->step; }

int orc_read_cell(const orc_ctx *o, uint32_t cell, uint8_t *species, double *vel, uint16_t *levels) {
  if (!o || cell >= o->n_cells) return E_INVAL;
  const cell_t *C = &o->cells[cell];
  uint32_t mm = o->max_modes;
  for (uint32_t i = 0; i < C->n; ++i) {
    species[i] = C->sp[i];
    vel[3 * i] = C->vx[i];
    vel[3 * i + 1] = C->vy[i];
    vel[3 * i + 2] = C->vz[i];
    for (uint32_t m = 0; m < mm; ++m) levels[(size_t)i * mm + m] = C->lvl[(size_t)i * mm + m];
  }
  return E_OK;
}

int orc_read_pos(const orc_ctx *o, uint32_t cell, double *pos) {
  if (!o || cell >= o->n_cells || !o->spatial) return E_INVAL;
  const cell_t *C = &o->cells[cell];
  for (uint32_t i = 0; i < C->n; ++i) {
    pos[3 * i] = C->px[i];
    pos[3 * i + 1] = C->py[i];
    pos[3 * i + 2] = C->pz[i];
  }
  return E_OK;
}

int orc_read_rot(const orc_ctx *o, uint32_t cell, double *rot) {
  if (!o || cell >= o->n_cells) return E_INVAL;
  const cell_t *C = &o->cells[cell];
  for (uint32_t i = 0; i < C->n; ++i) rot[i] = C->rot[i];
  return E_OK;
}

/* rotational energy of the cell's particles summed per species [J] */
int orc_rot_energy(const orc_ctx *o, uint32_t cell, double *per_species) {
  if (!o || cell >= o->n_cells) return E_INVAL;
  const cell_t *C = &o->cells[cell];
  for (uint32_t s = 0; s < o->n_species; ++s) per_species[s] = 0.0;
  for (uint32_t i = 0; i < C->n; ++i) per_species[C->sp[i]] += C->rot[i];
  return E_OK;
}

int orc_read_cell_state(const orc_ctx *o, uint32_t cell, double *sgmax, double *rem, uint64_t *ctr) {
  if (!o || cell >= o->n_cells) return E_INVAL;
  const cell_t *C = &o->cells[cell];
  *sgmax = C->sgmax;
  *rem = C->rem;
  memcpy(ctr, C->ctr, sizeof(C->ctr));
  return E_OK;
}

int orc_levels(const orc_ctx *o, uint32_t species, uint32_t mode, double *out, uint32_t max_n) {
  if (!o || species >= o->n_species) return E_INVAL;
  const species_t *s = &o->sp[species];
  if (mode >= s->n_modes) return E_INVAL;
  if (mode < s->n_bend) {
    for (uint32_t i = 0; i < max_n; ++i) out[i] = mode_energy(s, mode, i);
    return (int)max_n;
  }
  uint32_t n = s->idiss[mode] + 1;
  for (uint32_t i = 0; i < n && i < max_n; ++i) out[i] = s->lev[mode][i];
  return (int)n;
}

int orc_species_info(const orc_ctx *o, uint32_t species, double *zpe, uint32_t *n_modes, uint32_t *sampler) {
  if (!o || species >= o->n_species) return E_INVAL;
  *zpe = o->sp[species].zpe;
  *n_modes = o->sp[species].n_modes;
  *sampler = (uint32_t)o->sp[species].sampler;
  return E_OK;
}

int orc_pair_info(const orc_ctx *o, uint32_t a, uint32_t b, double *out8) {
  if (!o || !o->finalized || a >= o->n_species || b >= o->n_species) return E_INVAL;
  const pair_t *p = &o->pr[a][b];
  out8[0] = p->mr;
  out8[1] = p->hm;
  out8[2] = p->msum;
  out8[3] = p->wa;
  out8[4] = p->wb;
  out8[5] = p->csg;
  out8[6] = p->esg;
  out8[7] = p->q;
  return E_OK;
}

/* Per-cell moments, plain sequential sums in slot order:
 * out[0..2] sum m v, out[3] sum m |v|^2, out[4] total mass,
 * out[5] sum of formation energies,
 * then per species s: out[6+3s] count, out[7+3s] sum E_vib (with zero point),
 * out[8+3s] sum (E_vib - ZPE). */
int orc_moments(const orc_ctx *o, uint32_t cell, double *out) {
  if (!o || cell >= o->n_cells) return E_INVAL;
  const cell_t *C = &o->cells[cell];
  uint32_t mm = o->max_modes;
  memset(out, 0, sizeof(double) * (6 + 3 * o->n_species));
  for (uint32_t i = 0; i < C->n; ++i) {
    const species_t *S = &o->sp[C->sp[i]];
    double m = S->mass;
    out[0] += m * C->vx[i];
    out[1] += m * C->vy[i];
    out[2] += m * C->vz[i];
    out[3] += m * ((C->vx[i] * C->vx[i] + C->vy[i] * C->vy[i]) + C->vz[i] * C->vz[i]);
    out[4] += m;
    out[5] += S->formation;
    double ev = vib_energy(S, C->lvl + (size_t)i * mm);
    out[6 + 3 * C->sp[i]] += 1.0;
    out[7 + 3 * C->sp[i]] += ev;
    out[8 + 3 * C->sp[i]] += ev - S->zpe;
  }
  return E_OK;
}

/* Mean vibrational energy above the ground state at temperature t
 * (mean-energy equation of the implementation section). */
static double mean_evib(const species_t *s, double t) {
  double e = 0.0;
  for (uint32_t m = 0; m < s->n_bend; ++m) e += s->kt[m] / (exp(s->theta[m] / t) - 1.0);
  for (uint32_t m = s->n_bend; m < s->n_modes; ++m) {
    double num = 0.0, den = 0.0;
    for (uint32_t i = 0; i <= s->idiss[m]; ++i) {
      double de = s->lev[m][i] - s->lev[m][0];
      double w = exp(-de / (K_BOLTZ * t));
      num += de * w;
      den += w;
    }
    e += num / den;
  }
  return e;
}

/* T_vib by bisection in log T on [1, 1e6] K (zero-point search of the paper). */
int orc_tvib(const orc_ctx *o, uint32_t species, double target, double *t_out) {
  if (!o || species >= o->n_species) return E_INVAL;
  const species_t *s = &o->sp[species];
  if (s->n_modes == 0 || !(target > 0.0)) {
    *t_out = 0.0;
    return E_OK;
  }
  double lo = log(1.0), hi = log(1.0e6);
  if (mean_evib(s, exp(hi)) < target) {
    *t_out = exp(hi);
    return E_OK;
  }
  for (int it = 0; it < 200; ++it) {
    double mid = 0.5 * (lo + hi);
    if (mean_evib(s, exp(mid)) < target)
      lo = mid;
    else
      hi = mid;
    if (hi - lo < 1e-15) break;
  }
  *t_out = exp(0.5 * (lo + hi));
  return E_OK;
}

/* ------------------------------------------------------------------ */
/* Single-operation drivers                                              */
/* ------------------------------------------------------------------ */
/* n independent relaxations of one species; item i uses stream
 * (pair = i, cell = 0xFFFFFFF0, step = current step). */
int orc_relax_batch(orc_ctx *o, uint32_t species, double q, int sampler, uint32_t n, const double *e_tr,
                    const uint16_t *lvl_in, uint16_t *lvl_out, double *e_tr_out, uint64_t *trials) {
  if (!o || !o->finalized || species >= o->n_species) return E_INVAL;
  species_t s = o->sp[species];
  if (sampler == ORC_SAMPLER_JOINT || sampler == ORC_SAMPLER_GIBBS || sampler == ORC_SAMPLER_EXACT) s.sampler = sampler;
  uint32_t nm = s.n_modes;
  for (uint32_t i = 0; i < n; ++i) {
    stream st;
    stream_open(&st, o->seed, i, 0xFFFFFFF0u, o->step);
    uint16_t lv[ORC_MAX_MODES];
    for (uint32_t m = 0; m < nm; ++m) lv[m] = lvl_in[(size_t)i * nm + m];
    double et = e_tr[i];
    int capped;
    uint64_t t = relax(o, &s, lv, &et, q, &st, &capped);
    for (uint32_t m = 0; m < nm; ++m) lvl_out[(size_t)i * nm + m] = lv[m];
    e_tr_out[i] = et;
    if (trials) trials[i] = t;
  }
  return E_OK;
}

/* Heat-bath chain: iteration i draws nothing but the relaxation; the
 * translational energy offered to the molecule is the input e_tr[i].
 * Chain c uses streams (pair = i, cell = 0xFFFFFFF1, step = c).
 * hist[m * stride + level] counts the post-collision level of mode m
 * (hist may be NULL). */
int orc_relax_chain(orc_ctx *o, uint32_t species, double q, int sampler, uint32_t chain, uint32_t n_iter,
                    const double *e_tr, uint16_t *lvl_state, uint64_t *hist, uint32_t hist_stride) {
  if (!o || !o->finalized || species >= o->n_species) return E_INVAL;
  species_t s = o->sp[species];
  if (sampler == ORC_SAMPLER_JOINT || sampler == ORC_SAMPLER_GIBBS || sampler == ORC_SAMPLER_EXACT) s.sampler = sampler;
  for (uint32_t i = 0; i < n_iter; ++i) {
    stream st;
    stream_open(&st, o->seed, i, 0xFFFFFFF1u, chain);
    double et = e_tr[i];
    int capped;
    relax(o, &s, lvl_state, &et, q, &st, &capped);
    if (!hist) continue;
    for (uint32_t m = 0; m < s.n_modes; ++m) {
      uint32_t l = lvl_state[m];
      if (l < hist_stride) hist[(size_t)m * hist_stride + l] += 1;
    }
  }
  return E_OK;
}

/* n independent accepted collisions of given pairs (no NTC, no acceptance
 * draw); item i uses stream (pair = i, cell = 0xFFFFFFF2, step = current).
 * Arrays: sp[2n], vel[6n], lvl[2n x max_modes]; outputs likewise; born_*
 * receive the newborn of item i (born_sp = 255 when none). */
static int collide_batch(orc_ctx *o, uint32_t n, const uint8_t *sp, const double *vel, const uint16_t *lvl,
                         uint8_t *sp_out, double *vel_out, uint16_t *lvl_out, int32_t *reaction_out,
                         uint8_t *born_sp, double *born_vel, uint16_t *born_lvl, const uint8_t *m_sp, double *m_vel,
                         double t_cell, double n_cell, const double *rot, double *rot_out, double *born_rot);

int orc_collide_batch(orc_ctx *o, uint32_t n, const uint8_t *sp, const double *vel, const uint16_t *lvl,
                      uint8_t *sp_out, double *vel_out, uint16_t *lvl_out, int32_t *reaction_out,
                      uint8_t *born_sp, double *born_vel, uint16_t *born_lvl) {
  return collide_batch(o, n, sp, vel, lvl, sp_out, vel_out, lvl_out, reaction_out, born_sp, born_vel, born_lvl, NULL,
                       NULL, 0.0, 0.0, NULL, NULL, NULL);
}

/* as orc_collide_batch, with rotational energies rot[2n] in, rot_out[2n] and
 * born_rot[n] out */
int orc_collide_rot_batch(orc_ctx *o, uint32_t n, const uint8_t *sp, const double *vel, const uint16_t *lvl,
                          const double *rot, uint8_t *sp_out, double *vel_out, uint16_t *lvl_out, double *rot_out,
                          int32_t *reaction_out, uint8_t *born_sp, double *born_vel, uint16_t *born_lvl,
                          double *born_rot) {
  return collide_batch(o, n, sp, vel, lvl, sp_out, vel_out, lvl_out, reaction_out, born_sp, born_vel, born_lvl, NULL,
                       NULL, 0.0, 0.0, rot, rot_out, born_rot);
}

/* as orc_collide_batch, with a third body per item (m_sp[n], m_vel[3n] in and
 * out) at cell temperature t_cell and number density n_cell; a recombined
 * item reports species 255 on its vanished side */
int orc_collide3_batch(orc_ctx *o, uint32_t n, const uint8_t *sp, const double *vel, const uint16_t *lvl,
                       uint8_t *sp_out, double *vel_out, uint16_t *lvl_out, int32_t *reaction_out,
                       uint8_t *born_sp, double *born_vel, uint16_t *born_lvl, const uint8_t *m_sp, double *m_vel,
                       double t_cell, double n_cell) {
  return collide_batch(o, n, sp, vel, lvl, sp_out, vel_out, lvl_out, reaction_out, born_sp, born_vel, born_lvl, m_sp,
                       m_vel, t_cell, n_cell, NULL, NULL, NULL);
}

static int collide_batch(orc_ctx *o, uint32_t n, const uint8_t *sp, const double *vel, const uint16_t *lvl,
                         uint8_t *sp_out, double *vel_out, uint16_t *lvl_out, int32_t *reaction_out,
                         uint8_t *born_sp, double *born_vel, uint16_t *born_lvl, const uint8_t *m_sp, double *m_vel,
                         double t_cell, double n_cell, const double *rot, double *rot_out, double *born_rot) {
  if (!o || !o->finalized) return E_INVAL;
  uint32_t mm = o->max_modes;
  for (uint32_t i = 0; i < n; ++i) {
    pair_state ps;
    memset(&ps, 0, sizeof(ps));
    for (int x = 0; x < 2; ++x) {
      if (sp[2 * i + x] >= o->n_species) return E_INVAL;
      ps.sp[x] = sp[2 * i + x];
      for (int k = 0; k < 3; ++k) ps.v[x][k] = vel[6 * i + 3 * x + k];
      for (uint32_t m = 0; m < mm; ++m) ps.lvl[x][m] = lvl[((size_t)2 * i + x) * mm + m];
      ps.rot[x] = rot ? rot[2 * i + x] : 0.0;
    }
    if (m_sp) {
      ps.has_m = 1;
      ps.sp_m = m_sp[i];
      for (int k = 0; k < 3; ++k) ps.v_m[k] = m_vel[3 * i + k];
      ps.t_cell = t_cell;
      ps.n_cell = n_cell;
    }
    double dx = ps.v[0][0] - ps.v[1][0], dy = ps.v[0][1] - ps.v[1][1], dz = ps.v[0][2] - ps.v[1][2];
    double g2 = (dx * dx + dy * dy) + dz * dz;
    stream st;
    stream_open(&st, o->seed, i, 0xFFFFFFF2u, o->step);
    newborn nb;
    memset(&nb, 0, sizeof(nb));
    reaction_out[i] = collide(o, &ps, g2, &st, NULL, &nb);
    if (m_sp)
      for (int k = 0; k < 3; ++k) m_vel[3 * i + k] = ps.v_m[k];
    for (int x = 0; x < 2; ++x) {
      sp_out[2 * i + x] = ps.dead[x] ? (uint8_t)255 : ps.sp[x];
      for (int k = 0; k < 3; ++k) vel_out[6 * i + 3 * x + k] = ps.v[x][k];
      for (uint32_t m = 0; m < mm; ++m) lvl_out[((size_t)2 * i + x) * mm + m] = ps.lvl[x][m];
      if (rot_out) rot_out[2 * i + x] = ps.dead[x] ? 0.0 : ps.rot[x];
    }
    if (born_rot) born_rot[i] = nb.born ? nb.rot : 0.0;
    born_sp[i] = nb.born ? nb.sp : 255;
    for (int k = 0; k < 3; ++k) born_vel[3 * i + k] = nb.born ? nb.v[k] : 0.0;
    for (uint32_t m = 0; m < mm; ++m) born_lvl[(size_t)i * mm + m] = nb.born ? nb.lvl[m] : 0;
  }
  return E_OK;
}
